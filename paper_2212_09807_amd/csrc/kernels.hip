// kernels.hip -- gfx950 kernels of the pixelated-LArTPC charge path (arXiv 2212.09807, Sec. 3).
//
// Stage map (one event, or a batch of events whose pixel spaces are concatenated):
//   k_quench_drift   Sec. 3.1-3.2: recombination, lifetime, diffusion widths per segment; charge box in
//                    (tick, sub-pixel bin) space; pixel rectangle the box reaches; per-pixel pair counts (a
//                    difference array over the pixel grid, k_prefix_rows / k_prefix_cols).
//   scans            pair / cell offsets (exclusive scans), active-pixel compaction (slots).
//   k_fill_pairs     pixel-major (pixel, segment) pair lists; k_sort_pairs orders each list by segment id.
//   k_cells          Sec. 3.3.2 eq. (rho), expectation over the Gaussian perturbations: charge per
//                    (tick, x-bin, y-bin) cell of each segment, as a sum over sample points of separable
//                    truncated-Gaussian bin masses.
//   k_induce_*       Sec. 3.3.2 eq. (current): per (segment, pixel) pair and tick, the cells in the pixel's table
//                    reach convolved in time with the field-response column of their mirror-folded bin; summed
//                    over the pixel's segments (Sec. 3.4) either in a fixed order with Kahan compensation
//                    (sorted variant) or with FP32 atomics (atomic variant).
//   k_sum_*          the same sum by linearity as sum-then-convolve: segments' charges summed per sub-pixel
//                    column (column lists, sort, intervals, summed charges), per-pixel records by folded table
//                    column, the mirror merge, then k_induce_summed4 / k_induce_summed over the records.
//   k_electronics    Sec. 3.4: integrate, threshold (with discriminator noise), hold, digitise, reset, with
//                    Philox4x32-10 noise; also the FP64 per-event sum of the currents.
//   k_compact        packets of all pixels into the caller's arrays.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"
#include "launch.hpp"

namespace ltsim {

constexpr uint64_t kMask40 = (1ull << 40) - 1;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// FP64 per-event report accumulation, aggregated over the wavefront when all valid lanes share the event.
// Must be reached by all 64 lanes of the wavefront.
__device__ __forceinline__ void add_report(double *rep, int e, int k, double v, bool valid) {
    unsigned long long m = __ballot(valid);
    if (m == 0) return;
    int lead = __ffsll((long long)m) - 1;
    int el = __shfl(e, lead);
    bool same = __all(!valid || e == el);
    if (same) {
        double x = valid ? v : 0.0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lane_id() == lead && x != 0.0) atomicAdd(&rep[(int64_t)el * 5 + k], x);
    } else if (valid && v != 0.0) {
        atomicAdd(&rep[(int64_t)e * 5 + k], v);
    }
}

__device__ __forceinline__ int find_event(const int64_t *off, int n_ev, int64_t s) {
    int lo = 0, hi = n_ev - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= s) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ================================================================================================= scans
// Exclusive scan of int64 / uint64 arrays: per-tile reduce, scan of tile sums (one workgroup), per-tile scan.
constexpr int kScanPT = 8;
constexpr int kScanTile = kWG * kScanPT;

template <typename T>
__device__ __forceinline__ T block_exclusive(T v, T *lds, T &total) {
    // wavefront inclusive scan
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int i = 0; i < kWG / 64; ++i) { T t = lds[i]; lds[i] = run; run += t; }
        lds[kWG / 64] = run;
    }
    __syncthreads();
    T res = x - v + lds[wv];
    total = lds[kWG / 64];
    __syncthreads();
    return res;
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_scan_reduce(const T *data, int64_t n, T *part) {
    __shared__ T lds[kWG / 64 + 1];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPT;
    T s = 0;
#pragma unroll
    for (int i = 0; i < kScanPT; ++i)
        if (base + i < n) s += data[base + i];
    T tot;
    block_exclusive<T>(s, lds, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_scan_partials(T *part, int64_t nb) {
    __shared__ T lds[kWG / 64 + 1];
    T carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kWG) {
        int64_t i = b0 + threadIdx.x;
        T v = i < nb ? part[i] : 0;
        T tot;
        T ex = block_exclusive<T>(v, lds, tot);
        if (i < nb) part[i] = ex + carry;
        carry += tot;
    }
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_scan_apply(T *data, int64_t n, const T *part) {
    __shared__ T lds[kWG / 64 + 1];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPT;
    T v[kScanPT];
    T s = 0;
#pragma unroll
    for (int i = 0; i < kScanPT; ++i) {
        v[i] = base + i < n ? data[base + i] : 0;
        s += v[i];
    }
    T tot;
    T run = block_exclusive<T>(s, lds, tot) + part[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanPT; ++i)
        if (base + i < n) { data[base + i] = run; run += v[i]; }
}

int64_t scan_tmp_needed(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

template <typename T>
static void scan_exclusive(T *data, int64_t n, void *tmp, hipStream_t st) {
    if (n <= 0) return;
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    T *part = (T *)tmp;
    k_scan_reduce<T><<<(unsigned)nb, kWG, 0, st>>>(data, n, part);
    k_scan_partials<T><<<1, kWG, 0, st>>>(part, nb);
    k_scan_apply<T><<<(unsigned)nb, kWG, 0, st>>>(data, n, part);
}

void scan_exclusive_i64(int64_t *data, int64_t n, int64_t *, void *tmp, hipStream_t st) {
    scan_exclusive<int64_t>(data, n, tmp, st);
}
void scan_exclusive_u64(uint64_t *data, int64_t n, void *tmp, hipStream_t st) {
    scan_exclusive<unsigned long long>((unsigned long long *)data, n, tmp, st);
}

// ================================================================================================= quench / drift
struct QDOut {
    float q_r, q_a, t_drift, sigma_t, sigma_time, dedx;
    int32_t n_points, flags;
};

// Recombination (Sec. 3.1) and drift (Sec. 3.2) of segment s, plus its local reference frame.
__device__ __forceinline__ void segment_setup(const DevParams &P, const SegArrays &S, int64_t s, SegInfo &g, QDOut &o) {
    const float x0 = S.x0[s], y0 = S.y0[s], z0 = S.z0[s], t0 = S.t0[s];
    const float x1 = S.x1[s], y1 = S.y1[s], z1 = S.z1[s], t1 = S.t1[s];
    const float E = S.energy[s];
    int32_t flags = 0;
    const float dx = __fsub_rn(x1, x0), dy = __fsub_rn(y1, y0), dz = __fsub_rn(z1, z0), dt = __fsub_rn(t1, t0);
    // number of sample points (integer decided in IEEE single precision, no contraction)
    const float L2 = __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
    const float L = __fsqrt_rn(L2);
    const float cN = ceilf(__fdiv_rn(L, P.step));
    const int32_t N = cN >= 1.0f ? (int32_t)fminf(cN, 1.0e8f) : 1;
    float dedx;
    if (L > 0.0f) dedx = __fdiv_rn(E, L);                         // constant within the segment (Sec. 2)
    else if (S.dedx && isfinite(S.dedx[s])) dedx = S.dedx[s];
    else { dedx = 0.0f; flags |= SEG_INVALID; }
    // finite, and small enough that bin / tick indices stay far from int32 limits (|coordinate| <= 1e6)
    const float cmax = fmaxf(fmaxf(fmaxf(fabsf(x0), fabsf(y0)), fmaxf(fabsf(z0), fabsf(t0))),
                             fmaxf(fmaxf(fabsf(x1), fabsf(y1)), fmaxf(fabsf(z1), fabsf(t1))));
    const bool fin = isfinite(x0) && isfinite(y0) && isfinite(z0) && isfinite(t0) && isfinite(x1) && isfinite(y1) &&
                     isfinite(z1) && isfinite(t1) && isfinite(E);       // (fmaxf would drop NaNs)
    if (!(fin && cmax <= 1.0e6f && E >= 0.0f)) flags |= SEG_INVALID;
    if (N > 65536) flags |= SEG_TOO_LONG;
    float R;
    if (P.recomb_model == 0) {
        R = P.birks_ab / (1.0f + P.birks_kb_eps * dedx);           // eq. (birks)
    } else {
        const float xi = P.box_beta_eps * dedx;                    // eq. (box)
        R = xi > 0.0f ? logf(P.box_alpha + xi) / xi : -1.0f;
        if (!(R >= 0.0f)) { R = 0.0f; flags |= SEG_BOX_CLAMP; }
    }
    const float qr = R * (E * P.inv_w_ion);
    const float zm = 0.5f * (z0 + z1);
    const float td = fabsf(zm - P.za_hi) * P.inv_vd_hi;            // eq. (drift) at the midpoint
    const float qa = qr * expf(-td * P.inv_lifetime);              // eq. (lifetime)
    const float sT = sqrtf(P.two_dt * td);                         // sigma = sqrt(2 D t)
    const float sL = sqrtf(P.two_dl * td) * P.inv_vd_hi;           // longitudinal, as time

    g.q_r = qr; g.q_a = qa; g.q_pt = qa / (float)N; g.t_drift = td;
    g.sigma_t = sT; g.sigma_time = sL; g.dedx = dedx;
    g.n_points = N;
    float qa_seg = qa;
    // local frame: reference bin / tick of the start point and exact offsets
    ref_offset(x0, 0.0f, P.x0_hi, P.x0_lo, P.b_hi, P.b_lo, g.u_ref, g.ox);
    ref_offset(y0, 0.0f, P.y0_hi, P.y0_lo, P.b_hi, P.b_lo, g.v_ref, g.oy);
    float zh, zl;
    two_sum(z0, -P.za_hi, zh, zl);
    zl = __fsub_rn(zl, P.za_lo);
    const float dh = fabsf(zh), dl = zh >= 0.0f ? zl : -zl;       // |z0 - z_anode| as hi + lo
    const float q = __fmul_rn(dh, P.inv_vd_hi);
    const float qe = __fadd_rn(fmaf(dh, P.inv_vd_hi, -q), __fadd_rn(__fmul_rn(dh, P.inv_vd_lo), __fmul_rn(dl, P.inv_vd_hi)));
    float vh, ve;
    two_sum(t0, q, vh, ve);
    ref_offset(vh, __fadd_rn(ve, qe), P.tb_hi, P.tb_lo, P.tick_hi, P.tick_lo, g.a_ref, g.ot);
    const float zz0 = __fsub_rn(z0, P.za_hi), zz1 = __fsub_rn(z1, P.za_hi);
    const bool straddle = (zz0 < 0.0f && zz1 > 0.0f) || (zz0 > 0.0f && zz1 < 0.0f);
    const float sg = (zz0 > 0.0f || (zz0 == 0.0f && zz1 >= 0.0f)) ? 1.0f : -1.0f;
    g.dx = dx; g.dy = dy; g.dz = dz; g.dt = dt; g.zz0 = zz0;
    g.dta = fmaf(sg * dz, P.inv_vd_hi, dt);
    if (straddle) flags |= SEG_STRADDLE;
    g.flags = flags;
    if (P.per_point && !(flags & (SEG_INVALID | SEG_TOO_LONG))) {
        // collected charge = sum of the points' charges; the box uses the widths of the point farthest from the
        // anode (the widest cloud), a superset of the points' own supports
        float sum = 0.0f, cmp = 0.0f;
        for (int32_t mu = 0; mu < N; ++mu) {
            float q, a, b;
            point_drift(g, P, mu, q, a, b);
            const float y = q - cmp, t = sum + y;
            cmp = (t - sum) - y;
            sum = t;
        }
        qa_seg = sum;
        g.q_a = sum;
        g.q_pt = sum / (float)N;
        const float tdm = fmaxf(fabsf(zz0), fabsf(zz1)) * P.inv_vd_hi;
        g.sigma_t = sqrtf(P.two_dt * tdm);
        g.sigma_time = sqrtf(P.two_dl * tdm) * P.inv_vd_hi;
    }
    o.q_r = qr; o.q_a = qa_seg; o.t_drift = td; o.sigma_t = sT; o.sigma_time = sL; o.dedx = dedx;
    o.n_points = N; o.flags = flags;
}

// Charge box (tick x bin x bin) that the truncated clouds of the sample points can reach, and the pixel
// rectangle whose table reach meets it.
__device__ __forceinline__ void segment_box(const DevParams &P, SegInfo &g) {
    float lx0, ly0, lt0, lx1, ly1, lt1;
    point_local(g, P, 0, lx0, ly0, lt0);
    point_local(g, P, g.n_points - 1, lx1, ly1, lt1);
    float tmin = fminf(lt0, lt1), tmax = fmaxf(lt0, lt1);
    if ((g.flags & SEG_STRADDLE) && !(g.flags & (SEG_TOO_LONG | SEG_INVALID))) {
        for (int32_t mu = 1; mu < g.n_points - 1; ++mu) {
            float a, b, t;
            point_local(g, P, mu, a, b, t);
            tmin = fminf(tmin, t);
            tmax = fmaxf(tmax, t);
        }
    }
    const float ext = P.nsig * g.sigma_t, ext_t = P.nsig * g.sigma_time;
    const int32_t ulo = (int32_t)floorf(__fdiv_rn(fminf(lx0, lx1) - ext, P.b_hi));
    const int32_t uhi = (int32_t)floorf(__fdiv_rn(fmaxf(lx0, lx1) + ext, P.b_hi));
    const int32_t vlo = (int32_t)floorf(__fdiv_rn(fminf(ly0, ly1) - ext, P.b_hi));
    const int32_t vhi = (int32_t)floorf(__fdiv_rn(fmaxf(ly0, ly1) + ext, P.b_hi));
    const int32_t alo = (int32_t)floorf(__fdiv_rn(tmin - ext_t, P.tick_hi));
    const int32_t ahi = (int32_t)floorf(__fdiv_rn(tmax + ext_t, P.tick_hi));
    g.u0 = g.u_ref + ulo; g.nu = uhi - ulo + 1;
    g.v0 = g.v_ref + vlo; g.nv = vhi - vlo + 1;
    g.a0 = g.a_ref + alo; g.na = ahi - alo + 1;
    g.na_pad = (g.na + P.cell_pad - 1) / P.cell_pad * P.cell_pad;
    if (!(g.nu >= 1 && g.nu <= kBoxMax && g.nv >= 1 && g.nv <= kBoxMax && g.na >= 1 && g.na <= kNaMax))
        g.flags |= SEG_TOO_LONG;
    // pixel ix reaches sub-pixel bins u in [ix*nsub + nsub/2 - bx, ix*nsub + nsub/2 + bx - 1]
    const int32_t h = P.nsub / 2;
    g.ix0 = max(ceil_div(g.u0 - h - P.bx + 1, P.nsub), 0);
    g.ix1 = min(floor_div(g.u0 + g.nu - 1 - h + P.bx, P.nsub), P.nx - 1);
    g.iy0 = max(ceil_div(g.v0 - h - P.by + 1, P.nsub), 0);
    g.iy1 = min(floor_div(g.v0 + g.nv - 1 - h + P.by, P.nsub), P.ny - 1);
    if (g.flags & (SEG_INVALID | SEG_TOO_LONG)) { g.ix1 = g.ix0 - 1; }
    g.n_pairs = (g.ix1 >= g.ix0 && g.iy1 >= g.iy0) ? (g.ix1 - g.ix0 + 1) * (g.iy1 - g.iy0 + 1) : 0;
}

__global__ __launch_bounds__(kWG) void k_quench_drift(DevParams P, SegArrays S, int64_t n_seg, const int64_t *ev_off,
                                                      int32_t n_ev, SegInfo *si, int64_t *cell_cnt, uint64_t *pix_cnt,
                                                      DevHeader *H, double *report) {
    const int64_t s = (int64_t)blockIdx.x * kWG + threadIdx.x;
    const bool valid = s < n_seg;
    SegInfo g = {};
    QDOut o;
    int e = 0;
    if (valid) {
        e = find_event(ev_off, n_ev, s);
        segment_setup(P, S, s, g, o);
        segment_box(P, g);
        g.event = e;
        si[s] = g;
        const bool skip = g.flags & (SEG_INVALID | SEG_TOO_LONG);
        cell_cnt[s] = skip ? 0 : (int64_t)g.nu * g.nv * g.na_pad;
        if (!skip) atomicAdd((unsigned long long *)&H->n_colseg, (unsigned long long)g.nu * g.nv);
        if (g.flags & SEG_INVALID) atomicOr(&H->status, ST_INVALID);
        if (g.flags & SEG_TOO_LONG) atomicOr(&H->status, ST_TOO_LONG);
        // pairs per pixel: the reach is a rectangle of the event's pixel grid, counted by a difference array (+1 at
        // its first corner, -1 / -1 / +1 one past it; prefix sums along the rows and down the columns follow)
        if (g.ix1 >= g.ix0 && g.iy1 >= g.iy0) {
            unsigned long long *pc = (unsigned long long *)pix_cnt + (int64_t)e * P.npx;
            const int32_t xb = g.ix1 + 1, yb = g.iy1 + 1;
            atomicAdd(&pc[g.iy0 * P.nx + g.ix0], 1ull);
            if (xb < P.nx) atomicAdd(&pc[g.iy0 * P.nx + xb], ~0ull);
            if (yb < P.ny) {
                atomicAdd(&pc[yb * P.nx + g.ix0], ~0ull);
                if (xb < P.nx) atomicAdd(&pc[yb * P.nx + xb], 1ull);
            }
        }
    }
    add_report(report, e, 0, valid ? (double)g.q_r : 0.0, valid);
    add_report(report, e, 1, valid ? (double)g.q_a : 0.0, valid);
}

// Mark active pixels (count > 0) in the high bits so one scan yields pair offsets and slot indices.
__global__ void k_mark_active(uint64_t *pix_cnt, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        uint64_t v = pix_cnt[i];
        pix_cnt[i] = v | (v ? (1ull << 40) : 0ull);
    }
}

__global__ void k_totals(const uint64_t *pix_off, int64_t n_gp, const int64_t *cell_off, int64_t n_seg, DevHeader *H) {
    uint64_t t = pix_off[n_gp];
    H->n_pairs = (int64_t)(t & kMask40);
    H->n_slots = (int64_t)(t >> 40);
    H->n_cells = cell_off[n_seg];
}

// inclusive prefix sums along each row of a set of grids (one wavefront per row of len values)
__global__ __launch_bounds__(kWG) void k_prefix_rows(int64_t *a, int64_t n_rows, int32_t len) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (kWG / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (row >= n_rows) return;
    int64_t *r = a + row * len, carry = 0;
    for (int32_t c0 = 0; c0 < len; c0 += 64) {
        int64_t x = c0 + lane < len ? r[c0 + lane] : 0;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t y = __shfl_up(x, d);
            if (lane >= d) x += y;
        }
        x += carry;
        if (c0 + lane < len) r[c0 + lane] = x;
        carry = __shfl(x, 63);
    }
}

// inclusive prefix sums down each column of n_ev grids of CU rows x CV values (thread per (grid, v); eight
// rows loaded ahead)
__global__ void k_prefix_cols(int64_t *a, int32_t n_ev, int32_t CU, int32_t CV) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_ev * CV) return;
    const int64_t ev = t / CV, v = t - ev * CV;
    int64_t *p = a + ev * CU * CV + v, run = 0;
    int32_t u = 0;
    for (; u + 8 <= CU; u += 8) {
        int64_t x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = p[(int64_t)(u + i) * CV];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            run += x[i];
            p[(int64_t)(u + i) * CV] = run;
        }
    }
    for (; u < CU; ++u) {
        run += p[(int64_t)u * CV];
        p[(int64_t)u * CV] = run;
    }
}

void launch_quench_drift(const DevParams &P, const SegArrays &S, const Work &w, hipStream_t st) {
    const int64_t n_gp = (int64_t)w.n_ev * P.npx;
    if (w.n_seg > 0)
        k_quench_drift<<<(unsigned)((w.n_seg + kWG - 1) / kWG), kWG, 0, st>>>(P, S, w.n_seg, w.seg_ev_off, w.n_ev, w.si,
                                                                            w.cell_off, w.pix_cnt, w.hdr, w.report);
    if (n_gp > 0) {
        const int64_t rows = (int64_t)w.n_ev * P.ny;
        k_prefix_rows<<<(unsigned)((rows + kWG / 64 - 1) / (kWG / 64)), kWG, 0, st>>>((int64_t *)w.pix_cnt, rows, P.nx);
        k_prefix_cols<<<(unsigned)(((int64_t)w.n_ev * P.nx + kWG - 1) / kWG), kWG, 0, st>>>((int64_t *)w.pix_cnt,
                                                                                           w.n_ev, P.ny, P.nx);
    }
    k_mark_active<<<(unsigned)((n_gp + kWG - 1) / kWG), kWG, 0, st>>>(w.pix_cnt, n_gp);
    scan_exclusive<unsigned long long>((unsigned long long *)w.pix_cnt, n_gp + 1, w.scan_tmp, st);
    scan_exclusive<int64_t>(w.cell_off, w.n_seg + 1, w.scan_tmp, st);
    k_totals<<<1, 1, 0, st>>>(w.pix_cnt, n_gp, w.cell_off, w.n_seg, w.hdr);
}

__global__ void k_stage_qd(DevParams P, SegArrays S, int64_t n, float *out_f, int32_t *out_i) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    SegInfo g = {};
    QDOut o;
    segment_setup(P, S, s, g, o);
    float *f = out_f + 6 * s;
    f[0] = o.q_r; f[1] = o.q_a; f[2] = o.t_drift; f[3] = o.sigma_t; f[4] = o.sigma_time; f[5] = o.dedx;
    out_i[2 * s] = o.n_points;
    out_i[2 * s + 1] = o.flags & (SEG_BOX_CLAMP | SEG_INVALID);
}

void launch_stage_quench_drift(const DevParams &P, const SegArrays &S, int64_t n, float *out_f, int32_t *out_i,
                               hipStream_t st) {
    if (n > 0) k_stage_qd<<<(unsigned)((n + kWG - 1) / kWG), kWG, 0, st>>>(P, S, n, out_f, out_i);
}

// ================================================================================================= slots / pairs
__global__ void k_slots(DevParams P, int64_t n_gp, const uint64_t *pix_off, int32_t *pix_slot, int32_t *slot_gp,
                        int64_t *slot_off, int32_t *pixel_id_out, const DevHeader *H, int64_t cap_slots) {
    int64_t gp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gp > n_gp) return;
    if (gp == n_gp) {
        int64_t ns = H->n_slots;
        if (ns <= cap_slots) slot_off[ns] = H->n_pairs;
        return;
    }
    uint64_t v = pix_off[gp], vn = pix_off[gp + 1];
    bool active = (vn >> 40) > (v >> 40);
    int64_t slot = (int64_t)(v >> 40);
    pix_slot[gp] = active ? (int32_t)slot : -1;
    if (active && slot < cap_slots) {
        slot_gp[slot] = (int32_t)gp;
        slot_off[slot] = (int64_t)(v & kMask40);
        if (pixel_id_out) pixel_id_out[slot] = (int32_t)(gp % P.npx);
    }
}

__global__ void k_event_pixel_offsets(int32_t n_ev, int32_t npx, const uint64_t *pix_off, int64_t *ev_pix_off) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e <= n_ev) ev_pix_off[e] = (int64_t)(pix_off[(int64_t)e * npx] >> 40);
}

void launch_slots(const DevParams &P, const Work &w, int32_t *pixel_id_out, int64_t *ev_pix_off, hipStream_t st) {
    const int64_t n_gp = (int64_t)w.n_ev * P.npx;
    k_slots<<<(unsigned)((n_gp + 1 + kWG - 1) / kWG), kWG, 0, st>>>(P, n_gp, w.pix_cnt, w.pix_slot, w.slot_gp,
                                                                   w.slot_off, pixel_id_out, w.hdr, INT64_MAX);
    if (ev_pix_off)
        k_event_pixel_offsets<<<(w.n_ev + 1 + kWG - 1) / kWG, kWG, 0, st>>>(w.n_ev, P.npx, w.pix_cnt, ev_pix_off);
}

// Also stores each segment's scanned charge-cell offset in its record (the scan runs after k_quench_drift); with
// pairs = null only that.
__global__ __launch_bounds__(kWG) void k_fill_pairs(DevParams P, SegInfo *si, int64_t n_seg, const int64_t *cell_off,
                                                    const uint64_t *pix_off, int32_t *cursor, int32_t *pairs) {
    int64_t s = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (s >= n_seg) return;
    si[s].cell_off = cell_off[s];
    if (!pairs) return;                                  // the summed induction needs no pair lists
    const SegInfo &g = si[s];
    const int64_t base = (int64_t)g.event * P.npx;
    for (int32_t iy = g.iy0; iy <= g.iy1; ++iy)
        for (int32_t ix = g.ix0; ix <= g.ix1; ++ix) {
            int64_t gp = base + iy * P.nx + ix;
            int64_t pos = (int64_t)(pix_off[gp] & kMask40) + atomicAdd(&cursor[gp], 1);
            pairs[pos] = (int32_t)s;
        }
}

// Zero fill by a kernel (a memset node recorded into a captured graph is avoided: the pipeline's launch sequence
// may be captured).
__global__ void k_zero_words(uint32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void k_store_u64(uint64_t *p, uint64_t v) { *p = v; }

void launch_store_u64(uint64_t *p, uint64_t v, hipStream_t st) { k_store_u64<<<1, 1, 0, st>>>(p, v); }

void launch_zero(void *p, int64_t bytes, hipStream_t st) {
    const int64_t n = bytes / 4;
    if (n <= 0) return;
    const int64_t g = std::min<int64_t>((n + kWG - 1) / kWG, 4096);
    k_zero_words<<<(unsigned)g, kWG, 0, st>>>((uint32_t *)p, n);
}

void launch_fill_pairs(const DevParams &P, const Work &w, hipStream_t st) {
    if (w.n_seg > 0)
        k_fill_pairs<<<(unsigned)((w.n_seg + kWG - 1) / kWG), kWG, 0, st>>>(P, w.si, w.n_seg, w.cell_off, w.pix_cnt,
                                                                          w.cursor, w.pairs_unsorted);
}

// Each pixel's segment list in ascending segment id (ids are unique within a list): rank = number of smaller ids.
constexpr int kSortLds = 4096;
__global__ __launch_bounds__(kWG) void k_sort_pairs(const int64_t *slot_off, const DevHeader *H, const int32_t *in,
                                                    int32_t *out) {
    __shared__ int32_t lds[kSortLds];
    const int64_t n_slots = H->n_slots;
    for (int64_t slot = blockIdx.x; slot < n_slots; slot += gridDim.x) {
        const int64_t off = slot_off[slot];
        const int32_t cnt = (int32_t)(slot_off[slot + 1] - off);
        const int32_t *src = in + off;
        if (cnt <= kSortLds) {
            for (int i = threadIdx.x; i < cnt; i += kWG) lds[i] = src[i];
            __syncthreads();
            for (int i = threadIdx.x; i < cnt; i += kWG) {
                int32_t v = lds[i], r = 0;
                for (int j = 0; j < cnt; ++j) r += lds[j] < v;
                out[off + r] = v;
            }
            __syncthreads();
        } else {
            for (int i = threadIdx.x; i < cnt; i += kWG) {
                int32_t v = src[i], r = 0;
                for (int j = 0; j < cnt; ++j) r += src[j] < v;
                out[off + r] = v;
            }
        }
    }
}

void launch_sort_pairs(const Work &w, int64_t n_slots_host, hipStream_t st) {
    int64_t g = n_slots_host < 1 ? 1 : (n_slots_host > 8192 ? 8192 : n_slots_host);
    k_sort_pairs<<<(unsigned)g, kWG, 0, st>>>(w.slot_off, w.hdr, w.pairs_unsorted, w.pairs);
}

// ================================================================================================= charge cells
constexpr int kCellLds = 6144;    // floats (24 KB: several workgroups per CU; long segments take several passes)

// Monte Carlo cells of one segment (the paper's estimator of eq. (rho) with M = P.mc_draws perturbations per point):
// every moved copy of a sample point adds one hit to the cell that contains it (integer counts, in LDS when the box
// fits, else in the cell buffer itself), then cell = hits * q / M.  Counts make the result independent of the order
// in which the workgroup's threads land their hits.
__device__ void mc_cells(const DevParams &P, const SegInfo &g, uint32_t seg, uint64_t event, float *out,
                         uint32_t *lds, int64_t ncell) {
    const int tid = threadIdx.x;
    const bool in_lds = ncell <= kCellLds;
    uint32_t *hist = in_lds ? lds : (uint32_t *)out;
    for (int64_t c = tid; c < ncell; c += kWG) hist[c] = 0u;
    __threadfence();
    __syncthreads();
    const uint32_t M = (uint32_t)P.mc_draws;
    const int64_t nd = (int64_t)g.n_points * M;
    for (int64_t d = tid; d < nd; d += kWG) {
        float lx, ly, lt, gx, gy, gt;
        point_local(g, P, (int32_t)(d / M), lx, ly, lt);
        mc_normals(P, seg, (uint32_t)d, event, gx, gy, gt);
        // the truncated cloud lies inside the box; the clamps only guard the memory
        const int32_t u = min(max(g.u_ref + local_bin(fmaf(g.sigma_t, gx, lx), P.b_hi, P.b_lo) - g.u0, 0), g.nu - 1);
        const int32_t v = min(max(g.v_ref + local_bin(fmaf(g.sigma_t, gy, ly), P.b_hi, P.b_lo) - g.v0, 0), g.nv - 1);
        const int32_t a =
            min(max(g.a_ref + local_bin(fmaf(g.sigma_time, gt, lt), P.tick_hi, P.tick_lo) - g.a0, 0), g.na - 1);
        atomicAdd(&hist[((int64_t)u * g.nv + v) * g.na_pad + a], 1u);
    }
    __threadfence();
    __syncthreads();
    const float w = __fdiv_rn(g.q_pt, (float)M);
    for (int64_t c = tid; c < ncell; c += kWG) {
        const uint32_t h = in_lds ? hist[c] : __hip_atomic_load(&hist[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        out[c] = (float)h * w;
    }
    __syncthreads();
}

// The charge box of one pass over np sample points as a matrix product on the FP32 matrix cores: with the point index
// m as the contraction, cells[(u, v)][a] = sum_m (fx[m][u] fy[m][v]) ft[m][a], times q (the point charge when every
// point carries the same charge, else 1: ft then already holds it).  16x16x4 MFMA tiles: rows are 16 (u, v) columns
// of the box, columns 16 ticks, each instruction takes 4 points (lane l gives A[l % 16][l / 16] = fx fy of its row's
// column at point l / 16 and B[l / 16][l % 16] = ft of that point at its tick).  Each wavefront of the workgroup takes
// 2 x 2 blocks of tiles in turn, so every A value serves two tiles and every B value two; out-of-box rows, ticks and
// points contribute zeros and are not written.  `first` writes the pass's sums, otherwise they are added.
typedef float floatx4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void cells_mfma(const float *fx, const float *fy, const float *ft, int32_t nu, int32_t nv,
                                           int32_t nap, int32_t np, float q, bool first, float *out) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int32_t ncol = nu * nv, tm = (ncol + 15) / 16, tn = (nap + 15) / 16;
    const int32_t bm = (tm + 1) / 2, bn = (tn + 1) / 2;
    const int32_t il = lane & 15, kl = lane >> 4;
    for (int32_t blk = wv; blk < bm * bn; blk += kWG / 64) {
        const int32_t mi0 = (blk / bn) * 2, nj0 = (blk % bn) * 2;
        int32_t cu[2], cv[2], ta[2];
        bool cok[2], tok[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int32_t c = (mi0 + t) * 16 + il;
            cok[t] = c < ncol;
            cu[t] = cok[t] ? c / nv : 0;
            cv[t] = cok[t] ? c - (c / nv) * nv : 0;
            ta[t] = (nj0 + t) * 16 + il;
            tok[t] = ta[t] < nap;
        }
        floatx4 D[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) D[i][j] = (floatx4){0.0f, 0.0f, 0.0f, 0.0f};
        for (int32_t m0 = 0; m0 < np; m0 += 4) {
            const int32_t m = m0 + kl;
            const bool mok = m < np;
            float A[2], B[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const bool ka = mok && cok[t], kb = mok && tok[t];
                const float x = fx[ka ? m * nu + cu[t] : 0], y = fy[ka ? m * nv + cv[t] : 0];
                A[t] = ka ? x * y : 0.0f;
                const float z = ft[kb ? m * nap + ta[t] : 0];
                B[t] = kb ? z : 0.0f;
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) D[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[i], B[j], D[i][j], 0, 0, 0);
        }
        // lane l holds rows 4 (l / 16) + r of each tile (a box column) at column l % 16 (a tick)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int32_t c = (mi0 + i) * 16 + 4 * kl + r, a = (nj0 + j) * 16 + il;
                    if (c < ncol && a < nap) {
                        const float v = D[i][j][r] * q;
                        float *o = out + (int64_t)c * nap + a;
                        if (first) *o = v; else *o += v;
                    }
                }
    }
}

__global__ __launch_bounds__(kWG) void k_cells(DevParams P, const SegInfo *si, int64_t n_seg, float *cells,
                                               const int64_t *seg_ev_off, const uint64_t *event_ids, double *report) {
    __shared__ float sm[kCellLds];
    __shared__ double red[kWG / 64];
    const int tid = threadIdx.x;
    for (int64_t s = blockIdx.x; s < n_seg; s += gridDim.x) {
        const SegInfo g = si[s];
        if (g.flags & (SEG_INVALID | SEG_TOO_LONG)) continue;
        const int32_t nu = g.nu, nv = g.nv, na = g.na, nap = g.na_pad, N = g.n_points;
        const int32_t row = nu + nv + nap, ne = nu + nv + na + 3;      // bins and bin edges of a point's three axes
        const int32_t pc = min(256, kCellLds / (row + ne + 6));
        float *fx = sm, *fy = sm + pc * nu, *ft = fy + pc * nv;
        float *tl = ft + pc * nap;                      // [point][edge]: the edge's tail, negated below the mean
        float *pl = tl + pc * ne;                       // [point][6]: local x, y, t, widths, charge
        const int64_t ncell = (int64_t)nu * nv * nap;
        float *out = cells + g.cell_off;
        if (P.mc_draws > 0)
            mc_cells(P, g, (uint32_t)(s - seg_ev_off[g.event]), event_ids[g.event], out, (uint32_t *)sm, ncell);
        for (int32_t mu0 = 0; mu0 < (P.mc_draws > 0 ? 0 : N); mu0 += pc) {
            const int32_t np = min(pc, N - mu0);
            // Per point and axis, the masses of consecutive bins (edges (k0 + j) * width from the reference edge)
            // of the point's Gaussian of width sigma, truncated at +-n sigma and renormalised, each taken as a
            // difference of tails on the side away from the mean.  Spread over the workgroup: each point's frame,
            // then every edge's tail, then every bin's mass from its two edges.
            for (int m = tid; m < np; m += kWG) {
                float q = 1.0f, sT = g.sigma_t, sL = g.sigma_time;
                point_local(g, P, mu0 + m, pl[6 * m], pl[6 * m + 1], pl[6 * m + 2]);
                if (P.per_point) point_drift(g, P, mu0 + m, q, sT, sL);
                pl[6 * m + 3] = sT;
                pl[6 * m + 4] = sL;
                pl[6 * m + 5] = q;
            }
            __syncthreads();
            for (int r = tid; r < np * ne; r += kWG) {
                const int32_t m = r / ne, k = r - m * ne;
                const int ax = k <= nu ? 0 : k <= nu + nv + 1 ? 1 : 2;
                const int32_t j = ax == 0 ? k : ax == 1 ? k - nu - 1 : k - nu - nv - 2;
                const float l = pl[6 * m + ax], sg = pl[6 * m + (ax == 2 ? 4 : 3)];
                const int32_t k0 = ax == 0 ? g.u0 - g.u_ref : ax == 1 ? g.v0 - g.v_ref : g.a0 - g.a_ref;
                const float wh = ax == 2 ? P.tick_hi : P.b_hi, wl = ax == 2 ? P.tick_lo : P.b_lo;
                float t = 0.0f;
                if (sg > 0.0f) {
                    const float kf = (float)(k0 + j);
                    const float e = __fadd_rn(fmaf(kf, wh, -l), __fmul_rn(kf, wl));
                    const float z = fminf(fmaxf(e * (1.0f / sg), -P.nsig), P.nsig);
                    t = tail(z);
                    if (!(z >= 0.0f)) t = -t;               // the sign bit keeps the side of the mean
                }
                tl[r] = t;
            }
            __syncthreads();
            for (int r = tid; r < np * row; r += kWG) {
                const int32_t m = r / row, k = r - m * row;
                const int ax = k < nu ? 0 : k < nu + nv ? 1 : 2;
                const int32_t j = ax == 0 ? k : ax == 1 ? k - nu : k - nu - nv;
                const int32_t eo = ax == 0 ? 0 : ax == 1 ? nu + 1 : nu + nv + 2;
                float mass = 0.0f;
                if (ax < 2 || j < na) {
                    const float sg = pl[6 * m + (ax == 2 ? 4 : 3)];
                    if (sg > 0.0f) {
                        // tmass only asks on which side of the mean each edge lies; an edge at z = 0 counted as
                        // above it gives the same value, (1 - 1/2) - ta = 1/2 - ta
                        const float a = tl[m * ne + eo + j], b = tl[m * ne + eo + j + 1];
                        mass = tmass(__builtin_signbit(a) ? -1.0f : 1.0f, fabsf(a), __builtin_signbit(b) ? -1.0f : 1.0f,
                                     fabsf(b), P.inv_norm);
                    } else {                            // no spread: all of the point in the bin that holds it
                        const float l = pl[6 * m + ax];
                        const float wh = ax == 2 ? P.tick_hi : P.b_hi;
                        const int32_t k0 = ax == 0 ? g.u0 - g.u_ref : ax == 1 ? g.v0 - g.v_ref : g.a0 - g.a_ref;
                        mass = j == (int32_t)floorf(__fdiv_rn(l, wh)) - k0 ? 1.0f : 0.0f;
                    }
                    if (ax == 2 && P.per_point) mass *= pl[6 * m + 5];   // per point: its charge rides on the time masses
                }
                float *dst = ax == 0 ? fx + m * nu : ax == 1 ? fy + m * nv : ft + m * nap;
                dst[j] = mass;
            }
            __syncthreads();
            cells_mfma(fx, fy, ft, nu, nv, nap, np, P.per_point ? 1.0f : g.q_pt, mu0 == 0, out);
            __syncthreads();
        }
        // charge whose cells lie outside the pixel grid
        const int32_t ug = P.nx * P.nsub, vg = P.ny * P.nsub;
        if (g.u0 < 0 || g.u0 + nu > ug || g.v0 < 0 || g.v0 + nv > vg) {
            double loc = 0.0;
            for (int64_t c = tid; c < ncell; c += kWG) {
                const int32_t uv = (int32_t)(c / nap);
                const int32_t v = g.v0 + uv % nv, u = g.u0 + uv / nv;
                if (u < 0 || u >= ug || v < 0 || v >= vg) loc += (double)out[c];
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) loc += __shfl_xor(loc, o);
            if (lane_id() == 0) red[tid >> 6] = loc;
            __syncthreads();
            if (tid == 0) {
                double t = 0.0;
                for (int i = 0; i < kWG / 64; ++i) t += red[i];
                if (t != 0.0) atomicAdd(&report[(int64_t)g.event * 5 + 4], t);
            }
            __syncthreads();
        }
    }
}

void launch_cells(const DevParams &P, const Work &w, hipStream_t st) {
    if (w.n_seg <= 0) return;
    int64_t g = w.n_seg > 8192 ? 8192 : w.n_seg;
    k_cells<<<(unsigned)g, kWG, 0, st>>>(P, w.si, w.n_seg, w.cells, w.seg_ev_off, w.event_ids, w.report);
}

// ================================================================================================= induction
// A global-memory pointer whose value is taken from the first active lane (wave-uniform by construction).  The
// global address space is kept explicit so loads through it stay global loads (a generic pointer would become a
// flat load, whose completion order forces a full wait on every outstanding load).
typedef const float __attribute__((address_space(1))) *gfloat_ptr;
__device__ __forceinline__ gfloat_ptr uniform_ptr(const float *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (gfloat_ptr)(((uint64_t)hi << 32) | lo);
}
// The same for data that no kernel of the launch writes (charge cells during induction): loads through the
// constant address space become scalar loads into SGPRs, read by the whole wavefront at once.
typedef const float __attribute__((address_space(4))) *cfloat_ptr;
__device__ __forceinline__ cfloat_ptr uniform_cptr(const float *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (cfloat_ptr)(((uint64_t)hi << 32) | lo);
}

// Current of one (segment, pixel) pair on RT consecutive ticks nb .. nb+RT-1 (eq. (current)):
//   I[n] = sum over cells (a, u, v) in the pixel's reach of c[a,u,v] * R[n - a + T_R - 1, fold(u - uc), fold(v - vc)].
// The table column is zero-padded by kPad on both sides, so no bounds test is needed in the inner loop; the cell
// column is padded with zeros to a multiple of kAC ticks.
template <int RT>
__device__ __forceinline__ void pair_block(const DevParams &P, const float *__restrict__ cc0, int32_t nv, int32_t nap,
                                           int32_t u0, int32_t v0, int32_t a0, const float *__restrict__ Rpad,
                                           int32_t ulo, int32_t uhi, int32_t vlo, int32_t vhi, int32_t uc, int32_t vc,
                                           int32_t nb, float (&acc)[RT]) {
    const int32_t K0 = nb - a0 + P.t_r - 1 + kPad;
    for (int32_t u = ulo; u <= uhi; ++u) {
        const int32_t i = fold(u - uc);
        const float *ccu = cc0 + (int64_t)(u - u0) * nv * nap;
        for (int32_t v = vlo; v <= vhi; ++v) {
            const int32_t j = fold(v - vc);
            const float *col = Rpad + (int64_t)(i * P.by + j) * P.col_len + K0 - (kAC - 1);
            const float *cc = ccu + (int64_t)(v - v0) * nap;
            for (int32_t ac = 0; ac < nap; ac += kAC) {
                float w[RT + kAC - 1];
#pragma unroll
                for (int m = 0; m < RT + kAC - 1; ++m) w[m] = col[m - ac];
                float cv[kAC];
#pragma unroll
                for (int q = 0; q < kAC; ++q) cv[q] = cc[ac + q];
#pragma unroll
                for (int q = 0; q < kAC; ++q)
#pragma unroll
                    for (int r = 0; r < RT; ++r) acc[r] = fmaf(cv[q], w[r - q + kAC - 1], acc[r]);
            }
        }
    }
}

// pair_block<8> with the loads of later cell-tick blocks (each a 15-value table window and 8 cell values) issued
// before the products of the current one, across column boundaries: the pair's blocks are walked as one sequence
// (column-major, all columns of a pair have the same number of blocks) with three register buffers in turn.
struct BlockCursor {
    int32_t u, v, j;
};

__device__ __forceinline__ void pair_block_pf(const DevParams &P, const float *__restrict__ cc0, int32_t nv, int32_t nap,
                                              int32_t u0, int32_t v0, int32_t a0, const float *__restrict__ Rpad,
                                              int32_t ulo, int32_t uhi, int32_t vlo, int32_t vhi, int32_t uc,
                                              int32_t vc, int32_t nb0, int32_t lane_off, float (&acc)[8]) {
    // table offset of the window's first value for the workgroup's first thread (uniform) and this thread's offset
    // from it (8 ticks per thread): every load is a uniform base plus a fixed 32-bit lane offset
    const int32_t K0w = nb0 - a0 + P.t_r - 1 + kPad - (kAC - 1);
    const int32_t nblk = nap / kAC;
    const int32_t total = (uhi - ulo + 1) * (vhi - vlo + 1) * nblk;
    BlockCursor f{ulo, vlo, 0};                         // next block to fetch
    int32_t nf = 0;                                     // blocks fetched so far
    // Loads are issued unconditionally (past the last block the last block is fetched again), so the number of
    // loads in flight is the same on every path and the waits only cover the block about to be used.
    auto fetch = [&](float (&w)[8 + kAC - 1], float (&cv)[kAC]) {
        const int64_t cb = (int64_t)(fold(f.u - uc) * P.by + fold(f.v - vc)) * P.col_len + K0w - kAC * f.j;
        gfloat_ptr base = (gfloat_ptr)(Rpad + cb);
        cfloat_ptr cc = (cfloat_ptr)(cc0 + ((int64_t)(f.u - u0) * nv + (f.v - v0)) * nap + kAC * f.j);
#pragma unroll
        for (int m = 0; m < 8 + kAC - 1; ++m) w[m] = base[lane_off + m];
#pragma unroll
        for (int q = 0; q < kAC; ++q) cv[q] = cc[q];
        if (++nf < total && ++f.j == nblk) {
            f.j = 0;
            if (++f.v > vhi) { f.v = vlo; ++f.u; }
        }
    };
    auto block = [&](const float (&w)[8 + kAC - 1], const float (&cv)[kAC]) {
#pragma unroll
        for (int q = 0; q < kAC; ++q)
#pragma unroll
            for (int r = 0; r < 8; ++r) acc[r] = fmaf(cv[q], w[r - q + kAC - 1], acc[r]);
    };
    // three register buffers in turn: the loads of block b + 2 are issued before the products of block b, so two
    // blocks of products cover each load's latency
    float wa[8 + kAC - 1], ca[kAC], wb[8 + kAC - 1], cb[kAC], wc[8 + kAC - 1], cx[kAC];
    fetch(wa, ca);
    fetch(wb, cb);
    for (int32_t b = 0; b < total; b += 3) {
        fetch(wc, cx);
        __builtin_amdgcn_sched_barrier(0);
        block(wa, ca);
        if (b + 1 >= total) break;
        fetch(wa, ca);
        __builtin_amdgcn_sched_barrier(0);
        block(wb, cb);
        if (b + 2 >= total) break;
        fetch(wb, cb);
        __builtin_amdgcn_sched_barrier(0);
        block(wc, cx);
    }
}

// Value of lane - 1 of the wavefront (DPP wave_shr:1); lane 0 has no source lane and keeps `lane0`.
__device__ __forceinline__ float shift_up_or(float v, float lane0) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, lane0),
                                                                  __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}


// The same product for RT = 8, streaming each table column through a ring of four 8-value register blocks.  Lane t
// covers ticks nb .. nb+7; for cell-tick block j (ticks a0 + 8j .. +7) its window is R[K0-8j-7 .. K0-8j+7], i.e.
// its block b_j = R[K0-8j .. +7] and seven values of b_{j+1} = R[K0-8j-8 .. -1], so every block serves two
// consecutive cell-tick blocks and is fetched once.  Block b_{j+3} is fetched into the slot of the dead block
// b_{j-1}, three blocks ahead; the next column's first three blocks are fetched while the current column runs.
//   Two ways to fetch b_{j+1}:
//   * SHIFT = false: every lane loads its own 8 values (two 16-byte loads when ALIGNED, i.e. K0 % 8 == 0);
//   * SHIFT = true: b_{j+1} is b_j of the lane below (DPP wave_shr:1); only lane 0 loads (its values come from
//     below the wavefront's span).  All 64 lanes must then execute the loop (inactive lanes get a safe in-bounds
//     base; their results are discarded, and lanes above an inactive lane are inactive too).
template <int S, bool SHIFT>
__device__ __forceinline__ void ring_block(float (&B)[4][8], const float (&cv)[kAC], float (&acc)[8]) {
    constexpr int N = (S + 1) & 3;
    if constexpr (SHIFT) {
#pragma unroll
        for (int k = 0; k < 8; ++k) B[N][k] = shift_up_or(B[S][k], B[N][k]);
    }
    // w[m] = R[K0 - 8j - 7 + m]: m < 7 from b_{j+1}[m + 1], m >= 7 from b_j[m - 7]
#pragma unroll
    for (int q = 0; q < kAC; ++q)
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int m = r - q + kAC - 1;
            acc[r] = fmaf(cv[q], m < 7 ? B[N][m + 1] : B[S][m - 7], acc[r]);
        }
}

template <bool ALIGNED>
__device__ __forceinline__ void load8(const float *p, float (&d)[8]) {
    if constexpr (ALIGNED) {
        const float4 a = *(const float4 *)p, b = *(const float4 *)(p + 4);
        d[0] = a.x; d[1] = a.y; d[2] = a.z; d[3] = a.w; d[4] = b.x; d[5] = b.y; d[6] = b.z; d[7] = b.w;
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) d[k] = p[k];
    }
}

// Streams a sequence of (table column, cell column) pairs through the ring.  `col` is this lane's pointer to
// R[K0 .. K0+7] of the first table column, `cc` the first cell column (nblk blocks of kAC ticks).  adv(col, cc, nblk)
// moves to the next column (false at the end); it is called while the current column runs, so the next column's
// first blocks are in flight before they are needed.  done() runs after each column's last block.  Loads reach at
// most 8 * nblk + 16 values below K0 (every caller keeps them inside the column's zero padding); the cell values of
// the block after a column's last lie in the next column or in the buffer's kCellSlack tail.
template <bool SHIFT, bool ALIGNED, class Adv, class Done>
__device__ __forceinline__ void column_stream(const float *col, const float *cc, int32_t nblk, Adv adv, Done done,
                                              float (&acc)[8]) {
    const bool lane0 = lane_id() == 0;
    gfloat_ptr col0 = uniform_ptr(col);
    float F[8], P1[8] = {}, P2[8] = {};
    load8<ALIGNED>(col, F);
    if (!SHIFT) {
        load8<ALIGNED>(col - 8, P1);
        load8<ALIGNED>(col - 16, P2);
    } else if (lane0) {                                 // lane 0 alone loads what is shifted in at the bottom
#pragma unroll
        for (int k = 0; k < 8; ++k) { P1[k] = col0[k - 8]; P2[k] = col0[k - 16]; }
    }
    const float *cl = col;
    for (;;) {
        float B[4][8];
#pragma unroll
        for (int k = 0; k < 8; ++k) { B[0][k] = F[k]; B[1][k] = P1[k]; B[2][k] = P2[k]; B[3][k] = 0.0f; }
        gfloat_ptr c0 = col0;
        const float *cur = cl;
        cfloat_ptr ccu = uniform_cptr(cc);
        const int32_t nb_cur = nblk;
        const bool more = adv(cl, cc, nblk);
        if (more) {                                     // next column, one column ahead
            col0 = uniform_ptr(cl);
            load8<ALIGNED>(cl, F);
            if (!SHIFT) {
                load8<ALIGNED>(cl - 8, P1);
                load8<ALIGNED>(cl - 16, P2);
            } else if (lane0) {
#pragma unroll
                for (int k = 0; k < 8; ++k) { P1[k] = col0[k - 8]; P2[k] = col0[k - 16]; }
            }
        }
        float cvb[2][kAC];                              // cell values of the current and the next block
#pragma unroll
        for (int q = 0; q < kAC; ++q) cvb[0][q] = ccu[q];
        for (int32_t j = 0; j < nb_cur; j += 4) {
#define LTS_RING_STEP(S)                                                                        \
    {                                                                                           \
        _Pragma("unroll") for (int q = 0; q < kAC; ++q) cvb[(S + 1) & 1][q] = ccu[kAC * (j + S + 1) + q]; \
        if constexpr (!SHIFT) {                                                                 \
            load8<ALIGNED>(cur - 8 * (j + S + 3), B[(S + 3) & 3]);                              \
        } else if (lane0) {                                                                     \
            _Pragma("unroll") for (int k = 0; k < 8; ++k) B[(S + 3) & 3][k] = c0[k - 8 * (j + S + 3)]; \
        }                                                                                       \
        __builtin_amdgcn_sched_barrier(0);          /* keep the prefetches ahead of this block's math */ \
        ring_block<S, SHIFT>(B, cvb[S & 1], acc);                                               \
    }
            LTS_RING_STEP(0)
            if (j + 1 >= nb_cur) break;
            LTS_RING_STEP(1)
            if (j + 2 >= nb_cur) break;
            LTS_RING_STEP(2)
            if (j + 3 >= nb_cur) break;
            LTS_RING_STEP(3)
#undef LTS_RING_STEP
        }
        done();
        if (!more) break;
    }
}

// Products of one table column with one cell column for RT = 8, two 8-value blocks in ping-pong: block j of cell
// ticks needs b_j = R[K0-8j .. +7] and b_{j+1} = R[K0-8j-8 .. -1]; the buffer holding b_j is refilled with b_{j+2}
// after block j, so each block loads only its 8 new values (no copies, no cross-lane traffic).
template <bool ALIGNED>
__device__ __forceinline__ void column_pingpong(const float *col, cfloat_ptr cc, int32_t nblk, float (&acc)[8]) {
    float X[8], Y[8], cv[kAC];
    load8<ALIGNED>(col, X);
    for (int32_t j = 0; j < nblk; j += 2) {
        load8<ALIGNED>(col - 8 * (j + 1), Y);
#pragma unroll
        for (int q = 0; q < kAC; ++q) cv[q] = cc[kAC * j + q];
#pragma unroll
        for (int q = 0; q < kAC; ++q)
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int m = r - q + kAC - 1;
                acc[r] = fmaf(cv[q], m < 7 ? Y[m + 1] : X[m - 7], acc[r]);
            }
        if (j + 1 >= nblk) break;
        load8<ALIGNED>(col - 8 * (j + 2), X);
#pragma unroll
        for (int q = 0; q < kAC; ++q) cv[q] = cc[kAC * (j + 1) + q];
#pragma unroll
        for (int q = 0; q < kAC; ++q)
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int m = r - q + kAC - 1;
                acc[r] = fmaf(cv[q], m < 7 ? X[m + 1] : Y[m - 7], acc[r]);
            }
    }
}


// One (segment, pixel) pair through the lane-exchange ring: the columns (u, v) of its charge box inside the pixel's
// reach, in row order.
__device__ __forceinline__ void pair_block_ring(const DevParams &P, const float *__restrict__ cc0, int32_t nv, int32_t nap,
                                                int32_t u0, int32_t v0, int32_t a0, const float *__restrict__ Rpad,
                                                int32_t ulo, int32_t uhi, int32_t vlo, int32_t vhi, int32_t uc,
                                                int32_t vc, int32_t nb, bool active, float (&acc)[8]) {
    const int32_t K0 = active ? nb - a0 + P.t_r - 1 + kPad : kPad;
    int32_t u = ulo, v = vlo;
    auto colp = [&](int32_t uu, int32_t vv) {
        return Rpad + (int64_t)(fold(uu - uc) * P.by + fold(vv - vc)) * P.col_len + K0;
    };
    auto cellp = [&](int32_t uu, int32_t vv) { return cc0 + ((int64_t)(uu - u0) * nv + (vv - v0)) * nap; };
    auto adv = [&](const float *&col, const float *&cc, int32_t &nblk) {
        if (++v > vhi) { v = vlo; ++u; }
        if (u > uhi) return false;
        col = colp(u, v);
        cc = cellp(u, v);
        return true;
    };
    column_stream<true, false>(colp(u, v), cellp(u, v), nap / kAC, adv, [] {}, acc);
}

// Signed induction of a pair's cells that falls outside the tick window [0, n_ticks), from FP64 prefix sums of
// the table columns.  Threads of the workgroup split the cells; returns this thread's part.
__device__ double pair_clipped(const DevParams &P, const float *cc0, int32_t nv, int32_t nap, int32_t na, int32_t u0,
                               int32_t v0, int32_t a0, const double *prefix, int32_t ulo, int32_t uhi, int32_t vlo,
                               int32_t vhi, int32_t uc, int32_t vc) {
    double acc = 0.0;
    const int32_t nuu = uhi - ulo + 1, nvv = vhi - vlo + 1;
    const int64_t tot = (int64_t)nuu * nvv * na;
    const int32_t T = P.t_r;
    for (int64_t c = threadIdx.x; c < tot; c += kWG) {
        const int32_t a = (int32_t)(c % na);
        const int32_t uv = (int32_t)(c / na);
        const int32_t v = vlo + uv % nvv, u = ulo + uv / nvv;
        const float cval = cc0[((int64_t)(u - u0) * nv + (v - v0)) * nap + a];
        if (cval == 0.0f) continue;
        const int32_t aa = a0 + a;
        const double *pf = prefix + (int64_t)(fold(u - uc) * P.by + fold(v - vc)) * (T + 1);
        const int32_t klo = min(max(T - 1 - aa, 0), T);                 // first kept table tick
        const int32_t khi = min(max(P.nticks + T - 1 - aa, 0), T);       // one past the last kept tick
        const double dropped = klo >= khi ? pf[T] : pf[klo] + (pf[T] - pf[khi]);
        acc += (double)cval * dropped;
    }
    return acc;
}

__device__ __forceinline__ double block_sum_double(double v, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if (lane_id() == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kWG / 64; ++i) t += red[i];
    return t;
}

// Sorted variant: one workgroup per active pixel (dynamic work queue); the pixel's segments in ascending id
// order; per-pair FP32 sums in registers added into a Kahan-compensated FP32 accumulator in LDS.
template <int RT, bool SHIFT, bool PREFETCH = false>
__global__ __launch_bounds__(kWG) void k_induce_sorted(DevParams P, const SegInfo *__restrict__ si,
                                                       const float *__restrict__ cells, const float *__restrict__ Rpad,
                                                       const double *__restrict__ prefix,
                                                       const int64_t *__restrict__ slot_off,
                                                       const int32_t *__restrict__ pairs,
                                                       const int32_t *__restrict__ slot_gp,
                                                       const int32_t *__restrict__ order, float *__restrict__ wave,
                                                       DevHeader *H, double *report) {
    extern __shared__ float sm[];
    __shared__ int32_t s_slot;
    __shared__ double red[kWG / 64];
    const int NT = P.nticks;
    float *s_sum = sm, *s_cmp = sm + NT;
    const int tid = threadIdx.x;
    const int64_t n_slots = H->n_slots;
    for (;;) {
        if (tid == 0) s_slot = (int32_t)atomicAdd(&H->work[0], 1u);
        __syncthreads();
        if (s_slot >= n_slots) break;
        const int64_t slot = order ? order[s_slot] : s_slot;           // largest-first when an order is given
        for (int n = tid; n < NT; n += kWG) { s_sum[n] = 0.0f; s_cmp[n] = 0.0f; }
        const int32_t gp = slot_gp[slot];
        const int32_t e = gp / P.npx, p = gp - e * P.npx;
        const int32_t ix = p % P.nx, iy = p / P.nx;
        const int32_t uc = ix * P.nsub + P.nsub / 2, vc = iy * P.nsub + P.nsub / 2;
        const int64_t pb = slot_off[slot], pe = slot_off[slot + 1];
        double clip = 0.0;
        __syncthreads();
        for (int64_t q = pb; q < pe; ++q) {
            const int32_t s = __builtin_amdgcn_readfirstlane(pairs[q]);
            const SegInfo &g = si[s];
            const int32_t u0 = g.u0, v0 = g.v0, a0 = g.a0, nv = g.nv, nap = g.na_pad, na = g.na;
            const int32_t ulo = max(u0, uc - P.bx), uhi = min(u0 + g.nu - 1, uc + P.bx - 1);
            const int32_t vlo = max(v0, vc - P.by), vhi = min(v0 + nv - 1, vc + P.by - 1);
            if (ulo > uhi || vlo > vhi) continue;
            const float *cc0 = cells + g.cell_off;
            const int32_t wlo = a0 - (P.t_r - 1), whi = a0 + na - 1;
            if (wlo < 0 || whi >= NT)
                clip += pair_clipped(P, cc0, nv, nap, na, u0, v0, a0, prefix, ulo, uhi, vlo, vhi, uc, vc);
            const int32_t lo = max(wlo, 0), hi = min(whi, NT - 1);
            for (int32_t nb0 = lo; nb0 <= hi; nb0 += kWG * RT) {
                const int32_t nb = nb0 + tid * RT;
                float acc[RT];
#pragma unroll
                for (int r = 0; r < RT; ++r) acc[r] = 0.0f;
                if constexpr (RT == 8 && SHIFT)
                    pair_block_ring(P, cc0, nv, nap, u0, v0, a0, Rpad, ulo, uhi, vlo, vhi, uc, vc, nb, nb <= hi, acc);
                else if constexpr (RT == 8 && PREFETCH) {
                    if (nb <= hi)
                        pair_block_pf(P, cc0, nv, nap, u0, v0, a0, Rpad, ulo, uhi, vlo, vhi, uc, vc, nb0, tid * RT,
                                      acc);
                } else if (nb <= hi)
                    pair_block<RT>(P, cc0, nv, nap, u0, v0, a0, Rpad, ulo, uhi, vlo, vhi, uc, vc, nb, acc);
#pragma unroll
                for (int r = 0; r < RT; ++r) {
                    const int32_t n = nb + r;
                    if (n <= hi) {                                       // Kahan: s_cmp holds the lost low part
                        const float y = acc[r] - s_cmp[n];
                        const float t = s_sum[n] + y;
                        s_cmp[n] = (t - s_sum[n]) - y;
                        s_sum[n] = t;
                    }
                }
            }
            __syncthreads();
        }
        float *wrow = wave + slot * NT;
        for (int n = tid; n < NT; n += kWG) wrow[n] = s_sum[n] - s_cmp[n];
        const double c = block_sum_double(clip, red);
        if (tid == 0 && c != 0.0) atomicAdd(&report[(int64_t)e * 5 + 3], c);
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------------ matrix-core form
// By eq. (current), a pair's current is I[n] = sum_a sum_col c[col][a] R[col][n - c0 - a] with c0 = a0 - (T_R - 1):
// a column's cell ticks a against its table column, shifted by a.  Summing over the columns first gives the matrix
// product Z[a][tau] = sum_col c[col][a] R[col][tau] (cell ticks x table ticks, contracted over the pair's columns),
// and then I[n] = sum_a Z[a][n - c0 - a], a sum along the anti-diagonals of Z.  The product runs on 32x32x2 FP32
// MFMA instructions (lane l gives A[l % 32][l / 32] = c[col k0 + l / 32][a] and B[l / 32][l % 32] =
// R[col k0 + l / 32][tau]): both operands are rows of 32 consecutive floats, and there is no padding beyond
// rounding the cell ticks to 32 and the columns to 2.  Each 32 x 64 block of Z goes through LDS for the
// anti-diagonal sums, which each lane adds to its wavefront's output ticks in a fixed order.
typedef float floatx16 __attribute__((ext_vector_type(16)));
constexpr int32_t kBufferWord3 = 0x00020000;    // raw 32-bit buffer descriptor word 3 (gfx9 family)
constexpr int32_t kZT = 64;                     // table ticks per block of Z
constexpr int32_t kZA = 32;                     // cell ticks per block of Z
constexpr int32_t kZS = kZT + 1;                // LDS row stride of a Z block
constexpr int32_t kZOut = 512;                  // output ticks per wavefront and pass
constexpr int32_t kZLds = kZA * kZS + kZOut;    // floats of LDS per wavefront

// One pair's contribution to ticks n_w .. n_w + 511, added to Ow (this wavefront's 512 output sums in LDS).
__device__ __forceinline__ void pair_zgemm(const DevParams &P, const float *__restrict__ cc0, int32_t nu, int32_t nv,
                                           int32_t nap, int32_t na, int32_t u0, int32_t v0, int32_t a0,
                                           __amdgpu_buffer_rsrc_t rt, int32_t ulo, int32_t uhi, int32_t vlo,
                                           int32_t vhi, int32_t uc, int32_t vc, int32_t n_w, float *Zb, float *Ow) {
    const int l = lane_id();
    const int32_t c0 = a0 - (P.t_r - 1);
    const int32_t nvv = vhi - vlo + 1, ncol = (uhi - ulo + 1) * nvv;
    // the descriptors must be wavefront-uniform (scalar registers)
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)uniform_ptr(cc0), (short)0, __builtin_amdgcn_readfirstlane(nu * nv * nap * 4), kBufferWord3);
    for (int32_t ab = 0; ab < na; ab += kZA) {
        // table ticks that reach this wavefront's outputs from cell ticks ab .. ab + 31
        const int32_t t_first = max(n_w - c0 - ab - (kZA - 1), 0);
        const int32_t t_last = min(n_w + kZOut - 1 - c0 - ab, P.t_r - 1);
        for (int32_t t0 = t_first; t0 <= t_last; t0 += kZT) {
            floatx16 D[2];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int r = 0; r < 16; ++r) D[nt][r] = 0.0f;
            // 32x32x2: lane l gives A[l % 32][l / 32] (cell tick ab + l % 32 of column k0 + l / 32) and
            // B[l / 32][l % 32] (table tick t0 + 32 nt + l % 32 of that column)
            const int32_t i32 = l & 31, h = l >> 5;
            // this lane's columns: k = h, h + 2, ... in row-major (u, v) order; a step of 2 moves du rows and dv
            // columns, plus at most one wrap; colc (the column's cell offset) follows incrementally
            int32_t k = h, uu = ulo + h / nvv, vv = vlo + h % nvv;
            const int32_t du = 2 / nvv, dv = 2 - du * nvv;
            int32_t colc = ((uu - u0) * nv + (vv - v0)) * nap;
            const int32_t step_c = (du * nv + dv) * nap, wrap_c = (nv - nvv) * nap;
            auto fetch = [&](float &A, float (&B)[2]) {
                const bool valid = k < ncol;
                const int32_t fu = uu - uc, fv = vv - vc;
                const int32_t bin = __mul24(fu ^ (fu >> 31), P.by) + (fv ^ (fv >> 31));   // fold(), 24-bit products
                const int32_t colr = __mul24(bin, P.col_len) + kPad + t0 + i32;
                const int32_t a = ab + i32;
                const bool in = valid && a < na;
                const float cv = __builtin_bit_cast(
                    float, __builtin_amdgcn_raw_buffer_load_b32(rc, 4 * (in ? colc + a : 0), 0, 0));
                A = in ? cv : 0.0f;
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
                    B[nt] = __builtin_bit_cast(
                        float, __builtin_amdgcn_raw_buffer_load_b32(rt, 4 * (valid ? colr + 32 * nt : 0), 0, 0));
                k += 2;
                vv += dv;
                uu += du;
                colc += step_c;
                const bool wrap = vv > vhi;
                vv = wrap ? vv - nvv : vv;
                uu = wrap ? uu + 1 : uu;
                colc = wrap ? colc + wrap_c : colc;
            };
            auto step = [&](float A, const float (&B)[2]) {
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) D[nt] = __builtin_amdgcn_mfma_f32_32x32x2f32(A, B[nt], D[nt], 0, 0, 0);
            };
            const int32_t ks2 = (ncol + 1) >> 1;
            float A0, B0[2], A1, B1[2], A2, B2[2];
            fetch(A0, B0);
            fetch(A1, B1);
            for (int32_t st = 0; st < ks2; st += 3) {
                fetch(A2, B2);
                __builtin_amdgcn_sched_barrier(0);
                step(A0, B0);
                __builtin_amdgcn_sched_barrier(0);
                fetch(A0, B0);
                __builtin_amdgcn_sched_barrier(0);
                step(A1, B1);
                __builtin_amdgcn_sched_barrier(0);
                fetch(A1, B1);
                __builtin_amdgcn_sched_barrier(0);
                step(A2, B2);
                __builtin_amdgcn_sched_barrier(0);
            }
            // Z block to LDS: 32x32 layout, lane l register r holds row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int r = 0; r < 16; ++r) Zb[(8 * (r >> 2) + 4 * h + (r & 3)) * kZS + 32 * nt + i32] = D[nt][r];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // anti-diagonal d = t + a' holds the block's part of tick n = t0 + c0 + ab + d
            // (a fixed trip count with clamped indices, so all 32 LDS reads of a diagonal are issued together)
#pragma unroll
            for (int32_t half = 0; half < 2; ++half) {
                const int32_t d = l + 64 * half;
                const int32_t o = t0 + c0 + ab + d - n_w;
                float sum = 0.0f;
#pragma unroll
                for (int32_t ap = 0; ap < kZA; ++ap) {
                    const int32_t t = d - ap;
                    const float z = Zb[ap * kZS + min(max(t, 0), kZT - 1)];
                    sum += (t >= 0 && t < kZT) ? z : 0.0f;
                }
                if (d < kZT + kZA - 1 && o >= 0 && o < kZOut) Ow[o] += sum;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// Per-pair induction of the sorted variant on the matrix cores: the same pixel-slot work queue, pair order and
// Kahan accumulation in LDS as k_induce_sorted; wavefront w of the workgroup owns ticks nb0 + 512 w .. + 511 of
// each 2048-tick pass over a pair's window, lane l of it ticks + 8 l .. + 7.
__global__ __launch_bounds__(kWG) void k_induce_mfma(DevParams P, const SegInfo *__restrict__ si,
                                                     const float *__restrict__ cells, const float *__restrict__ Rpad,
                                                     const double *__restrict__ prefix,
                                                     const int64_t *__restrict__ slot_off,
                                                     const int32_t *__restrict__ pairs,
                                                     const int32_t *__restrict__ slot_gp, float *__restrict__ wave,
                                                     DevHeader *H, double *report) {
    extern __shared__ float sm[];
    __shared__ int32_t s_slot;
    __shared__ double red[kWG / 64];
    const int NT = P.nticks;
    float *s_sum = sm, *s_cmp = sm + NT;
    const int tid = threadIdx.x;
    const int32_t wv = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;   // wavefront index (uniform)
    float *Zb = sm + 2 * NT + wv * kZLds, *Ow = Zb + kZA * kZS;
    const int64_t n_slots = H->n_slots;
    const __amdgpu_buffer_rsrc_t rt =
        __builtin_amdgcn_make_buffer_rsrc((void *)Rpad, (short)0, P.bx * P.by * P.col_len * 4, kBufferWord3);
    for (int o = l; o < kZOut; o += 64) Ow[o] = 0.0f;
    for (;;) {
        if (tid == 0) s_slot = (int32_t)atomicAdd(&H->work[0], 1u);
        __syncthreads();
        const int64_t slot = s_slot;
        if (slot >= n_slots) break;
        for (int n = tid; n < NT; n += kWG) { s_sum[n] = 0.0f; s_cmp[n] = 0.0f; }
        const int32_t gp = slot_gp[slot];
        const int32_t e = gp / P.npx, p = gp - e * P.npx;
        const int32_t ix = p % P.nx, iy = p / P.nx;
        const int32_t uc = ix * P.nsub + P.nsub / 2, vc = iy * P.nsub + P.nsub / 2;
        const int64_t pb = slot_off[slot], pe = slot_off[slot + 1];
        double clip = 0.0;
        __syncthreads();
        for (int64_t qq = pb; qq < pe; ++qq) {
            const int32_t s = __builtin_amdgcn_readfirstlane(pairs[qq]);
            const SegInfo &g = si[s];
            const int32_t u0 = g.u0, v0 = g.v0, a0 = g.a0, nv = g.nv, nap = g.na_pad, na = g.na;
            const int32_t ulo = max(u0, uc - P.bx), uhi = min(u0 + g.nu - 1, uc + P.bx - 1);
            const int32_t vlo = max(v0, vc - P.by), vhi = min(v0 + nv - 1, vc + P.by - 1);
            if (ulo > uhi || vlo > vhi) continue;
            const float *cc0 = cells + g.cell_off;
            const int32_t wlo = a0 - (P.t_r - 1), whi = a0 + na - 1;
            if (wlo < 0 || whi >= NT)
                clip += pair_clipped(P, cc0, nv, nap, na, u0, v0, a0, prefix, ulo, uhi, vlo, vhi, uc, vc);
            const int32_t lo = max(wlo, 0), hi = min(whi, NT - 1);
            for (int32_t nb0 = lo; nb0 <= hi; nb0 += 4 * kZOut) {
                const int32_t n_w = nb0 + kZOut * wv;
                if (n_w <= hi) {
                    pair_zgemm(P, cc0, g.nu, nv, nap, na, u0, v0, a0, rt, ulo, uhi, vlo, vhi, uc, vc, n_w, Zb, Ow);
#pragma unroll
                    for (int r = 0; r < 8; ++r) {
                        const int32_t o = 8 * l + r, n = n_w + o;
                        const float x = Ow[o];
                        Ow[o] = 0.0f;
                        if (n <= hi) {                                   // Kahan: s_cmp holds the lost low part
                            const float y = x - s_cmp[n];
                            const float z = s_sum[n] + y;
                            s_cmp[n] = (z - s_sum[n]) - y;
                            s_sum[n] = z;
                        }
                    }
                }
            }
            __syncthreads();
        }
        float *wrow = wave + slot * NT;
        for (int n = tid; n < NT; n += kWG) wrow[n] = s_sum[n] - s_cmp[n];
        const double c = block_sum_double(clip, red);
        if (tid == 0 && c != 0.0) atomicAdd(&report[(int64_t)e * 5 + 3], c);
        __syncthreads();
    }
}

// Atomic variant: one workgroup per segment (dynamic work queue); its pairs in pixel order; FP32 atomics.
template <int RT>
__global__ __launch_bounds__(kWG) void k_induce_atomic(DevParams P, const SegInfo *__restrict__ si, int64_t n_seg,
                                                       const float *__restrict__ cells, const float *__restrict__ Rpad,
                                                       const double *__restrict__ prefix,
                                                       const int32_t *__restrict__ pix_slot, float *wave, DevHeader *H,
                                                       double *report) {
    __shared__ int32_t s_seg;
    __shared__ double red[kWG / 64];
    const int NT = P.nticks;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s_seg = (int32_t)atomicAdd(&H->work[1], 1u);
        __syncthreads();
        const int64_t s = s_seg;
        __syncthreads();
        if (s >= n_seg) break;
        const SegInfo &g = si[s];
        if (g.n_pairs == 0) continue;
        const int32_t u0 = g.u0, v0 = g.v0, a0 = g.a0, nv = g.nv, nap = g.na_pad, na = g.na;
        const float *cc0 = cells + g.cell_off;
        const int32_t wlo = a0 - (P.t_r - 1), whi = a0 + na - 1;
        const int32_t lo = max(wlo, 0), hi = min(whi, NT - 1);
        double clip = 0.0;
        for (int32_t iy = g.iy0; iy <= g.iy1; ++iy)
            for (int32_t ix = g.ix0; ix <= g.ix1; ++ix) {
                const int32_t uc = ix * P.nsub + P.nsub / 2, vc = iy * P.nsub + P.nsub / 2;
                const int32_t ulo = max(u0, uc - P.bx), uhi = min(u0 + g.nu - 1, uc + P.bx - 1);
                const int32_t vlo = max(v0, vc - P.by), vhi = min(v0 + nv - 1, vc + P.by - 1);
                if (ulo > uhi || vlo > vhi) continue;
                const int64_t slot = pix_slot[(int64_t)g.event * P.npx + iy * P.nx + ix];
                float *wrow = wave + slot * NT;
                if (wlo < 0 || whi >= NT)
                    clip += pair_clipped(P, cc0, nv, nap, na, u0, v0, a0, prefix, ulo, uhi, vlo, vhi, uc, vc);
                for (int32_t nb0 = lo; nb0 <= hi; nb0 += kWG * RT) {
                    const int32_t nb = nb0 + tid * RT;
                    if (nb > hi) continue;
                    float acc[RT];
#pragma unroll
                    for (int r = 0; r < RT; ++r) acc[r] = 0.0f;
                    pair_block<RT>(P, cc0, nv, nap, u0, v0, a0, Rpad, ulo, uhi, vlo, vhi, uc, vc, nb, acc);
#pragma unroll
                    for (int r = 0; r < RT; ++r)
                        if (nb + r <= hi && acc[r] != 0.0f) atomicAdd(&wrow[nb + r], acc[r]);
                }
            }
        const double c = block_sum_double(clip, red);
        if (tid == 0 && c != 0.0) atomicAdd(&report[(int64_t)g.event * 5 + 3], c);
    }
}

// XCD-sliced sorted variant: workgroup b handles pixel slot slot0 + b / NS and slice x = b % NS of the
// mirror-folded x-bin index (table bins i in [x*bx/NS, (x+1)*bx/NS)).  Workgroups are dispatched to the 8 XCDs
// round-robin by id, so each XCD's L2 only ever holds its slice of the field-response table.  The pixel's per-slice
// waveform (Kahan over its segments in ascending order) goes to part[x][slot - slot0][tick]; k_sum_slices adds the
// slices in a fixed order.  Deterministic and batch-invariant like the unsliced kernel.
template <int RT>
__global__ __launch_bounds__(kWG) void k_induce_slices(DevParams P, int32_t NS, int64_t slot0, int64_t chunk,
                                                       const SegInfo *__restrict__ si, const float *__restrict__ cells,
                                                       const float *__restrict__ Rpad, const double *__restrict__ prefix,
                                                       const int64_t *__restrict__ slot_off,
                                                       const int32_t *__restrict__ pairs,
                                                       const int32_t *__restrict__ slot_gp, float *__restrict__ part,
                                                       const DevHeader *H, double *report) {
    extern __shared__ float sm[];
    __shared__ double red[kWG / 64];
    const int NT = P.nticks;
    float *s_sum = sm, *s_cmp = sm + NT;
    const int tid = threadIdx.x;
    const int64_t local = blockIdx.x / NS;
    const int32_t x = blockIdx.x - (int32_t)local * NS;
    const int64_t slot = slot0 + local;
    if (slot >= H->n_slots) return;
    const int32_t ilo = x * P.bx / NS, ihi = (x + 1) * P.bx / NS - 1;
    for (int n = tid; n < NT; n += kWG) { s_sum[n] = 0.0f; s_cmp[n] = 0.0f; }
    const int32_t gp = slot_gp[slot];
    const int32_t e = gp / P.npx, p = gp - e * P.npx;
    const int32_t ix = p % P.nx, iy = p / P.nx;
    const int32_t uc = ix * P.nsub + P.nsub / 2, vc = iy * P.nsub + P.nsub / 2;
    const int64_t pb = slot_off[slot], pe = slot_off[slot + 1];
    double clip = 0.0;
    __syncthreads();
    if (ilo <= ihi) {
        for (int64_t q = pb; q < pe; ++q) {
            const int32_t s = __builtin_amdgcn_readfirstlane(pairs[q]);
            const SegInfo &g = si[s];
            const int32_t u0 = g.u0, v0 = g.v0, a0 = g.a0, nv = g.nv, nap = g.na_pad, na = g.na;
            const int32_t ue = u0 + g.nu - 1;
            // fold(u - uc) in [ilo, ihi]: u - uc in [ilo, ihi] or in [-ihi-1, -ilo-1]
            const int32_t ua0 = max(u0, uc + ilo), ua1 = min(ue, uc + ihi);
            const int32_t ub0 = max(u0, uc - ihi - 1), ub1 = min(ue, uc - ilo - 1);
            const int32_t vlo = max(v0, vc - P.by), vhi = min(v0 + nv - 1, vc + P.by - 1);
            if ((ua0 > ua1 && ub0 > ub1) || vlo > vhi) continue;
            const float *cc0 = cells + g.cell_off;
            const int32_t wlo = a0 - (P.t_r - 1), whi = a0 + na - 1;
            if (wlo < 0 || whi >= NT) {
                if (ua0 <= ua1) clip += pair_clipped(P, cc0, nv, nap, na, u0, v0, a0, prefix, ua0, ua1, vlo, vhi, uc, vc);
                if (ub0 <= ub1) clip += pair_clipped(P, cc0, nv, nap, na, u0, v0, a0, prefix, ub0, ub1, vlo, vhi, uc, vc);
            }
            const int32_t lo = max(wlo, 0), hi = min(whi, NT - 1);
            for (int32_t nb0 = lo; nb0 <= hi; nb0 += kWG * RT) {
                const int32_t nb = nb0 + tid * RT;
                float acc[RT];
#pragma unroll
                for (int r = 0; r < RT; ++r) acc[r] = 0.0f;
                if (nb <= hi) {
                    if (ua0 <= ua1) pair_block<RT>(P, cc0, nv, nap, u0, v0, a0, Rpad, ua0, ua1, vlo, vhi, uc, vc, nb, acc);
                    if (ub0 <= ub1) pair_block<RT>(P, cc0, nv, nap, u0, v0, a0, Rpad, ub0, ub1, vlo, vhi, uc, vc, nb, acc);
                }
#pragma unroll
                for (int r = 0; r < RT; ++r) {
                    const int32_t n = nb + r;
                    if (n <= hi) {
                        const float y = acc[r] - s_cmp[n];
                        const float t = s_sum[n] + y;
                        s_cmp[n] = (t - s_sum[n]) - y;
                        s_sum[n] = t;
                    }
                }
            }
            __syncthreads();
        }
    }
    float *prow = part + ((int64_t)x * chunk + local) * NT;
    for (int n = tid; n < NT; n += kWG) prow[n] = s_sum[n] - s_cmp[n];
    const double c = block_sum_double(clip, red);
    if (tid == 0 && c != 0.0) atomicAdd(&report[(int64_t)e * 5 + 3], c);
}

// current[slot][n] = sum over slices x = 0..NS-1 (in that order, Kahan) of part[x][slot - slot0][n].
__global__ __launch_bounds__(kWG) void k_sum_slices(int32_t NS, int32_t NT, int64_t slot0, int64_t chunk,
                                                    const float *__restrict__ part, float *__restrict__ wave,
                                                    const DevHeader *H) {
    const int64_t n_slots = H->n_slots;
    const int64_t nrows = min(chunk, n_slots - slot0);
    const int64_t total = nrows * NT;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < total; i += (int64_t)gridDim.x * kWG) {
        float sum = 0.0f, cmp = 0.0f;
        for (int32_t x = 0; x < NS; ++x) {
            const float y = part[(int64_t)x * chunk * NT + i] - cmp;
            const float t = sum + y;
            cmp = (t - sum) - y;
            sum = t;
        }
        wave[slot0 * NT + i] = sum - cmp;
    }
}

// Largest-first order of the active pixels for the per-pair induction.  A workgroup owns one pixel at a time and
// takes the next from a counter, so pixels of very unequal work taken in pixel order leave the chip idle at the end
// while the last heavy pixels finish; taking them largest first (bucketed by the logarithm of their work, 16 buckets
// per octave) keeps the tail short.  Work of a pixel = sum over its pairs of the charge-box columns in its reach times
// the cell-tick blocks.  The order changes only which workgroup computes a pixel, not any sum.
__global__ void k_slot_work(DevParams P, const SegInfo *__restrict__ si, const int64_t *__restrict__ slot_off,
                            const int32_t *__restrict__ pairs, const int32_t *__restrict__ slot_gp, int64_t n_slots,
                            int32_t *__restrict__ bucket, int32_t *__restrict__ hist) {
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= n_slots) return;
    const int32_t gp = slot_gp[slot];
    const int32_t p = gp % P.npx;
    const int32_t uc = (p % P.nx) * P.nsub + P.nsub / 2, vc = (p / P.nx) * P.nsub + P.nsub / 2;
    double work = 0.0;
    for (int64_t q = slot_off[slot]; q < slot_off[slot + 1]; ++q) {
        const SegInfo &g = si[pairs[q]];
        const int32_t cu = min(g.u0 + g.nu, uc + P.bx) - max(g.u0, uc - P.bx);
        const int32_t cv = min(g.v0 + g.nv, vc + P.by) - max(g.v0, vc - P.by);
        if (cu > 0 && cv > 0) work += (double)cu * cv * (g.na_pad / kAC);
    }
    const int32_t lg = work >= 1.0 ? (int32_t)(16.0 * log2(work)) : 0;
    const int32_t b = kOrderBuckets - 1 - min(lg, kOrderBuckets - 1);          // descending work
    bucket[slot] = b;
    atomicAdd(&hist[b], 1);
}

// bucket offsets (exclusive scan of the histogram) into the cursors
__global__ void k_order_offsets(int32_t *__restrict__ hist, int32_t *__restrict__ cursor) {
    __shared__ int32_t s[kOrderBuckets];
    for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x) s[i] = hist[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int i = 0; i < kOrderBuckets; ++i) {
            const int32_t c = s[i];
            s[i] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x) cursor[i] = s[i];
}

__global__ void k_order_scatter(const int32_t *__restrict__ bucket, int64_t n_slots, int32_t *__restrict__ cursor,
                                int32_t *__restrict__ order) {
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= n_slots) return;
    order[atomicAdd(&cursor[bucket[slot]], 1)] = (int32_t)slot;
}

// w.order holds [order: n_slots][bucket: n_slots][hist: kOrderBuckets][cursor: kOrderBuckets]
static void launch_slot_order(const DevParams &P, const Work &w, int64_t n_slots, hipStream_t st) {
    int32_t *order = w.order, *bucket = order + n_slots, *hist = bucket + n_slots, *cursor = hist + kOrderBuckets;
    launch_zero(hist, (int64_t)sizeof(int32_t) * kOrderBuckets, st);
    const unsigned g = (unsigned)((n_slots + kWG - 1) / kWG);
    k_slot_work<<<g, kWG, 0, st>>>(P, w.si, w.slot_off, w.pairs, w.slot_gp, n_slots, bucket, hist);
    k_order_offsets<<<1, kWG, 0, st>>>(hist, cursor);
    k_order_scatter<<<g, kWG, 0, st>>>(bucket, n_slots, cursor, order);
}

template <int RT>
static void induce_slices_rt(const DevParams &P, const Work &w, const Table &T, float *wave, int64_t n_slots, int32_t NS,
                             float *part, int64_t chunk, hipStream_t st) {
    const size_t lds = (size_t)2 * P.nticks * sizeof(float);
    for (int64_t s0 = 0; s0 < n_slots; s0 += chunk) {
        const int64_t rows = n_slots - s0 < chunk ? n_slots - s0 : chunk;
        k_induce_slices<RT><<<(unsigned)(rows * NS), kWG, lds, st>>>(P, NS, s0, chunk, w.si, w.cells, T.Rpad, T.prefix,
                                                                   w.slot_off, w.pairs, w.slot_gp, part, w.hdr, w.report);
        int64_t g = (rows * P.nticks + kWG - 1) / kWG;
        if (g > 16384) g = 16384;
        k_sum_slices<<<(unsigned)g, kWG, 0, st>>>(NS, P.nticks, s0, chunk, part, wave, w.hdr);
    }
}

// Ticks per thread of the induction: the smallest of 1, 2, 4, 8 whose 256-thread tile covers a pair's window
// (table length + a typical charge-box extent), unless forced.
static int32_t pick_rt(const DevParams &P, int32_t forced) {
    if (forced == 1 || forced == 2 || forced == 4 || forced == 8) return forced;
    const int32_t win = P.t_r + 32;
    return win <= kWG ? 1 : win <= 2 * kWG ? 2 : win <= 4 * kWG ? 4 : 8;
}

void launch_induce_slices(const DevParams &P, const Work &w, const Table &T, float *wave, int64_t n_slots, int32_t NS,
                          float *part, int64_t chunk, int32_t rt, hipStream_t st) {
    if (n_slots <= 0) return;
    switch (pick_rt(P, rt)) {
        case 1: induce_slices_rt<1>(P, w, T, wave, n_slots, NS, part, chunk, st); break;
        case 2: induce_slices_rt<2>(P, w, T, wave, n_slots, NS, part, chunk, st); break;
        case 4: induce_slices_rt<4>(P, w, T, wave, n_slots, NS, part, chunk, st); break;
        default: induce_slices_rt<8>(P, w, T, wave, n_slots, NS, part, chunk, st); break;
    }
}

template <int RT, bool SHIFT, bool PREFETCH = false>
static void induce_rt(const DevParams &P, const Work &w, const Table &T, float *wave, int mode, int64_t n_slots,
                      hipStream_t st) {
    const int64_t cap = 2048;
    if (mode == 0) {
        int64_t g = n_slots < 1 ? 1 : (n_slots > cap ? cap : n_slots);
        size_t lds = (size_t)2 * P.nticks * sizeof(float);
        if (w.order && n_slots > 0) launch_slot_order(P, w, n_slots, st);
        k_induce_sorted<RT, SHIFT, PREFETCH><<<(unsigned)g, kWG, lds, st>>>(P, w.si, w.cells, T.Rpad, T.prefix, w.slot_off, w.pairs,
                                                          w.slot_gp, n_slots > 0 ? w.order : nullptr, wave, w.hdr,
                                                          w.report);
    } else {
        int64_t g = w.n_seg < 1 ? 1 : (w.n_seg > cap ? cap : w.n_seg);
        k_induce_atomic<RT><<<(unsigned)g, kWG, 0, st>>>(P, w.si, w.n_seg, w.cells, T.Rpad, T.prefix, w.pix_slot, wave,
                                                        w.hdr, w.report);
    }
}

void launch_induce_mfma(const DevParams &P, const Work &w, const Table &T, float *wave, int64_t n_slots,
                        hipStream_t st) {
    const int64_t cap = 2048;
    const int64_t g = n_slots < 1 ? 1 : (n_slots > cap ? cap : n_slots);
    const size_t lds = ((size_t)2 * P.nticks + (size_t)(kWG / 64) * kZLds) * sizeof(float);
    k_induce_mfma<<<(unsigned)g, kWG, lds, st>>>(P, w.si, w.cells, T.Rpad, T.prefix, w.slot_off, w.pairs, w.slot_gp,
                                                  wave, w.hdr, w.report);
}

void launch_induce(const DevParams &P, const Work &w, const Table &T, float *wave, int mode, int64_t n_slots, int32_t rt,
                   bool shift, hipStream_t st) {
    switch (pick_rt(P, rt)) {
        case 1: induce_rt<1, false>(P, w, T, wave, mode, n_slots, st); break;
        case 2: induce_rt<2, false>(P, w, T, wave, mode, n_slots, st); break;
        case 4: induce_rt<4, false>(P, w, T, wave, mode, n_slots, st); break;
        default:
            if (shift) induce_rt<8, true>(P, w, T, wave, mode, n_slots, st);
            else if (rt == 0) induce_rt<8, false, true>(P, w, T, wave, mode, n_slots, st);   // auto: prefetched
            else induce_rt<8, false>(P, w, T, wave, mode, n_slots, st);
            break;
    }
}

// ================================================================================================= stage hooks
// The paper's own data flow (Sec. 3.3.2, 3.4): the induced current of every (segment, pixel) pair is materialised as
// its own waveform, then the waveforms of each pixel are summed.  The fused kernels above never write these; the
// hooks below do, for tests and for comparison with the fused path.

// Pair list in stored order (pixel-major, ascending segment within a pixel): segment index and tile pixel id.
__global__ __launch_bounds__(kWG) void k_pair_list(DevParams P, const int64_t *__restrict__ slot_off,
                                                   const int32_t *__restrict__ pairs,
                                                   const int32_t *__restrict__ slot_gp, const DevHeader *H,
                                                   int32_t *pair_seg, int32_t *pair_pix) {
    for (int64_t slot = blockIdx.x; slot < H->n_slots; slot += gridDim.x) {
        const int32_t gp = slot_gp[slot];
        const int32_t p = gp - (gp / P.npx) * P.npx;
        for (int64_t q = slot_off[slot] + threadIdx.x; q < slot_off[slot + 1]; q += kWG) {
            if (pair_seg) pair_seg[q] = pairs[q];
            if (pair_pix) pair_pix[q] = p;
        }
    }
}

// Row q of `out` (n_ticks floats) receives pair q's current I_sp[n]: workgroup per active pixel, its pairs in
// stored order; ticks outside the pair's reach in time are written as zero.
template <int RT>
__global__ __launch_bounds__(kWG) void k_induce_pairs(DevParams P, const SegInfo *__restrict__ si,
                                                      const float *__restrict__ cells, const float *__restrict__ Rpad,
                                                      const int64_t *__restrict__ slot_off,
                                                      const int32_t *__restrict__ pairs,
                                                      const int32_t *__restrict__ slot_gp, const DevHeader *H,
                                                      float *__restrict__ out) {
    const int NT = P.nticks;
    const int tid = threadIdx.x;
    for (int64_t slot = blockIdx.x; slot < H->n_slots; slot += gridDim.x) {
        const int32_t gp = slot_gp[slot];
        const int32_t p = gp - (gp / P.npx) * P.npx;
        const int32_t ix = p % P.nx, iy = p / P.nx;
        const int32_t uc = ix * P.nsub + P.nsub / 2, vc = iy * P.nsub + P.nsub / 2;
        for (int64_t q = slot_off[slot]; q < slot_off[slot + 1]; ++q) {
            const SegInfo &g = si[__builtin_amdgcn_readfirstlane(pairs[q])];
            const int32_t u0 = g.u0, v0 = g.v0, a0 = g.a0, nv = g.nv, nap = g.na_pad, na = g.na;
            const int32_t ulo = max(u0, uc - P.bx), uhi = min(u0 + g.nu - 1, uc + P.bx - 1);
            const int32_t vlo = max(v0, vc - P.by), vhi = min(v0 + nv - 1, vc + P.by - 1);
            const bool any = ulo <= uhi && vlo <= vhi;
            const int32_t lo = any ? max(a0 - (P.t_r - 1), 0) : NT, hi = any ? min(a0 + na - 1, NT - 1) : -1;
            float *row = out + q * NT;
            for (int n = tid; n < NT; n += kWG)
                if (n < lo || n > hi) row[n] = 0.0f;
            const float *cc0 = cells + g.cell_off;
            for (int32_t nb0 = lo; nb0 <= hi; nb0 += kWG * RT) {
                const int32_t nb = nb0 + tid * RT;
                if (nb > hi) continue;
                float acc[RT];
#pragma unroll
                for (int r = 0; r < RT; ++r) acc[r] = 0.0f;
                pair_block<RT>(P, cc0, nv, nap, u0, v0, a0, Rpad, ulo, uhi, vlo, vhi, uc, vc, nb, acc);
#pragma unroll
                for (int r = 0; r < RT; ++r)
                    if (nb + r <= hi) row[nb + r] = acc[r];
            }
        }
    }
}

void launch_pair_list(const DevParams &P, const Work &w, int64_t n_slots, int32_t *pair_seg, int32_t *pair_pix,
                      hipStream_t st) {
    if (n_slots <= 0) return;
    const unsigned g = (unsigned)std::min<int64_t>(n_slots, 65536);
    k_pair_list<<<g, kWG, 0, st>>>(P, w.slot_off, w.pairs, w.slot_gp, w.hdr, pair_seg, pair_pix);
}

void launch_induce_pairs(const DevParams &P, const Work &w, const Table &T, int64_t n_slots, float *out,
                         hipStream_t st) {
    if (n_slots <= 0) return;
    const unsigned g = (unsigned)std::min<int64_t>(n_slots, 65536);
    switch (pick_rt(P, 0)) {
        case 1: k_induce_pairs<1><<<g, kWG, 0, st>>>(P, w.si, w.cells, T.Rpad, w.slot_off, w.pairs, w.slot_gp, w.hdr, out); break;
        case 2: k_induce_pairs<2><<<g, kWG, 0, st>>>(P, w.si, w.cells, T.Rpad, w.slot_off, w.pairs, w.slot_gp, w.hdr, out); break;
        case 4: k_induce_pairs<4><<<g, kWG, 0, st>>>(P, w.si, w.cells, T.Rpad, w.slot_off, w.pairs, w.slot_gp, w.hdr, out); break;
        default: k_induce_pairs<8><<<g, kWG, 0, st>>>(P, w.si, w.cells, T.Rpad, w.slot_off, w.pairs, w.slot_gp, w.hdr, out); break;
    }
}

// Per-pixel sum of pair waveforms grouped by pixel: head[q] = 1 where a run of equal pixel ids starts (q < n),
// head[n] = 0; a pixel id below its predecessor sets ST_INVALID (the pairs are not grouped in ascending order).
__global__ void k_run_heads(const int32_t *__restrict__ pix, int64_t n, int64_t *head, DevHeader *H) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q > n) return;
    if (q == n) { head[q] = 0; return; }
    const int32_t prev = q > 0 ? pix[q - 1] : -1;
    head[q] = pix[q] != prev ? 1 : 0;
    if (pix[q] < prev) atomicOr(&H->status, ST_INVALID);
}

// After the exclusive scan of head: start[k] = first pair of run k, start[n_runs] = n; pixel ids of the runs.
__global__ void k_run_starts(const int32_t *__restrict__ pix, int64_t n, const int64_t *__restrict__ idx,
                             int64_t *start, int32_t *pixel_out, int64_t cap) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int64_t k = idx[q];
    if (q == 0 || pix[q] != pix[q - 1]) {
        start[k] = q;
        if (k < cap) pixel_out[k] = pix[q];
    }
    if (q == n - 1) start[idx[n]] = n;
}

// current[k][t] = sum over the run's pairs, in stored order, of their waveforms at tick t (Kahan summation).
__global__ __launch_bounds__(kWG) void k_reduce_runs(const float *__restrict__ pair_current,
                                                     const int64_t *__restrict__ start, int32_t NT, float *current) {
    const int64_t k = blockIdx.x;
    const int32_t t = blockIdx.y * kWG + threadIdx.x;
    if (t >= NT) return;
    float sum = 0.0f, cmp = 0.0f;
    for (int64_t q = start[k]; q < start[k + 1]; ++q) {
        const float y = pair_current[q * NT + t] - cmp;
        const float z = sum + y;
        cmp = (z - sum) - y;
        sum = z;
    }
    current[k * NT + t] = sum - cmp;
}

void launch_run_heads(const int32_t *pix, int64_t n, int64_t *head, DevHeader *H, hipStream_t st) {
    k_run_heads<<<(unsigned)((n + 1 + kWG - 1) / kWG), kWG, 0, st>>>(pix, n, head, H);
}

void launch_run_starts(const int32_t *pix, int64_t n, const int64_t *idx, int64_t *start, int32_t *pixel_out,
                       int64_t cap, hipStream_t st) {
    if (n > 0) k_run_starts<<<(unsigned)((n + kWG - 1) / kWG), kWG, 0, st>>>(pix, n, idx, start, pixel_out, cap);
}

void launch_reduce_runs(const float *pair_current, const int64_t *start, int64_t n_runs, int32_t NT, float *current,
                        hipStream_t st) {
    if (n_runs <= 0 || NT <= 0) return;
    const dim3 g((unsigned)n_runs, (unsigned)((NT + kWG - 1) / kWG));
    k_reduce_runs<<<g, kWG, 0, st>>>(pair_current, start, NT, current);
}

// ================================================================================================= summed induction
// Sum-then-convolve: by linearity of eq. (current), the current on pixel p is the time convolution of each absolute
// sub-pixel column's charge, summed over all segments, with that column's folded table column.  The columns are
// summed once per event (fixed segment order, Kahan) and cut into pieces of at most kPieceTicks ticks; each piece is
// a 1 x 1 x L charge box, and every active pixel's list of pieces in its reach replaces its pair list, so the
// sorted induction kernel runs unchanged on the summed data.

// Sort key of a segment in a column's list: first tick (signed, order-preserving bias) above the segment index.
__device__ __forceinline__ uint64_t sum_key(int32_t a0, int32_t s) {
    return ((uint64_t)((uint32_t)a0 ^ 0x80000000u) << 32) | (uint32_t)s;
}
__device__ __forceinline__ int32_t key_seg(uint64_t k) { return (int32_t)(uint32_t)k; }

// Segments per column.  A segment's reachable columns form a rectangle of the event's column grid, so the counts
// come from a two-dimensional difference array: per segment +1 at the rectangle's first corner and -1 / -1 / +1 at the
// corners one past it (those outside the grid dropped), then prefix sums along each row and down each grid column.
__global__ void k_sum_ranges(DevParams P, const SegInfo *si, int64_t n_seg, SumWork sw) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_seg) return;
    const SegInfo &g = si[s];
    if (g.flags & (SEG_INVALID | SEG_TOO_LONG)) return;
    sw.segc[s] = SumSeg{g.a0, g.na, g.u0, g.v0, g.nv, g.na_pad, g.cell_off};
    const int32_t u_a = max(g.u0, sw.UL), u_b = min(g.u0 + g.nu - 1, sw.UL + sw.CU - 1);
    const int32_t v_a = max(g.v0, sw.VL), v_b = min(g.v0 + g.nv - 1, sw.VL + sw.CV - 1);
    if (u_a > u_b || v_a > v_b) return;
    unsigned long long *cnt = (unsigned long long *)sw.col_seg_off + (int64_t)g.event * sw.CU * sw.CV;
    const int32_t ua = u_a - sw.UL, ub = u_b - sw.UL + 1, va = v_a - sw.VL, vb = v_b - sw.VL + 1;
    atomicAdd(&cnt[(int64_t)ua * sw.CV + va], 1ull);
    if (vb < sw.CV) atomicAdd(&cnt[(int64_t)ua * sw.CV + vb], ~0ull);          // -1
    if (ub < sw.CU) {
        atomicAdd(&cnt[(int64_t)ub * sw.CV + va], ~0ull);
        if (vb < sw.CV) atomicAdd(&cnt[(int64_t)ub * sw.CV + vb], 1ull);
    }
}

void launch_sum_ranges(const DevParams &P, const Work &w, const SumWork &sw, hipStream_t st) {
    if (w.n_seg > 0) k_sum_ranges<<<(unsigned)((w.n_seg + kWG - 1) / kWG), kWG, 0, st>>>(P, w.si, w.n_seg, sw);
    const int64_t n_ev = sw.n_cols / ((int64_t)sw.CU * sw.CV);
    const int64_t rows = n_ev * sw.CU;
    if (rows > 0) {
        k_prefix_rows<<<(unsigned)((rows + kWG / 64 - 1) / (kWG / 64)), kWG, 0, st>>>(sw.col_seg_off, rows, sw.CV);
        k_prefix_cols<<<(unsigned)((n_ev * sw.CV + kWG - 1) / kWG), kWG, 0, st>>>(sw.col_seg_off, (int32_t)n_ev, sw.CU,
                                                                                  sw.CV);
    }
}

// per segment (one wavefront, lanes over its reachable columns: every atomic instruction meets distinct cursors)
__global__ __launch_bounds__(kWG) void k_sum_fill(DevParams P, const SegInfo *si, int64_t n_seg, SumWork sw) {
    const int lane = threadIdx.x & 63;
    const int64_t s = (int64_t)blockIdx.x * (kWG / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (s >= n_seg) return;
    const SegInfo &g = si[s];
    if (g.flags & (SEG_INVALID | SEG_TOO_LONG)) return;
    const int32_t u_a = max(g.u0, sw.UL), u_b = min(g.u0 + g.nu - 1, sw.UL + sw.CU - 1);
    const int32_t v_a = max(g.v0, sw.VL), v_b = min(g.v0 + g.nv - 1, sw.VL + sw.CV - 1);
    if (u_a > u_b || v_a > v_b) return;
    const int32_t wv = v_b - v_a + 1, nc = (u_b - u_a + 1) * wv;
    const int64_t base = (int64_t)g.event * sw.CU * sw.CV + (int64_t)(u_a - sw.UL) * sw.CV + (v_a - sw.VL);
    const uint64_t key = sum_key(g.a0, (int32_t)s);
    for (int32_t i = lane; i < nc; i += 64) {
        const int32_t du = i / wv;
        const int64_t c = base + (int64_t)du * sw.CV + (i - du * wv);
        sw.col_tmp[sw.col_seg_off[c] + atomicAdd(&sw.col_cursor[c], 1)] = key;
    }
}

// A column's charge is cut where none of its segments has charge for more than kSumGap ticks: the zero ticks of
// such a gap would otherwise be convolved with the whole table column.  A new piece costs less than ~16 zero ticks.
constexpr int32_t kSumGap = 16;

// Pieces of kPieceTicks ticks of an interval of L ticks, and their summed-charge length (the last one padded to kAC).
__device__ inline void sum_interval_size(int32_t L, int64_t &np, int64_t &ns) {
    np = (L + kPieceTicks - 1) / kPieceTicks;
    const int32_t last = L - (int32_t)(np - 1) * kPieceTicks;
    ns = (np - 1) * kPieceTicks + (last + kAC - 1) / kAC * kAC;
}

// 64-bit value of lane j (j wave-uniform).
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int j) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}

// per column: sort its segment list by key (first tick, segment index) into col_seg, then count the pieces and the
// padded summed-charge length of its merged tick intervals.  For the 512-tick summed induction kernel every
// interval's first tick is moved down to the residue it chooses (it makes every lane's table offsets aligned there);
// the 256-tick kernel takes intervals as they are (align_res < 0).  The order depends only on the segments' charge
// boxes and their order within the event, so the sums are the same in a batch and alone.  The columns with segments
// are listed first (k_sum_active); persistent wavefronts take them one at a time.  Sort by ranks (a key's place is
// the number of smaller keys; keys are unique): lane i holds key i of a 64-key chunk and compares it with every key
// of the list, taken chunk by chunk from the lanes' registers.  Intervals from the sorted list, 64 entries at a time:
// an entry starts an interval when its first tick lies more than kSumGap ticks beyond the last tick of every earlier
// entry (a prefix maximum over the lanes), and the interval before it ends at that maximum.
__device__ __forceinline__ int32_t key_a0(uint64_t k) { return (int32_t)((uint32_t)(k >> 32) ^ 0x80000000u); }
__device__ __forceinline__ void interval_count(int32_t lo, int32_t hi, int32_t res, int64_t &np, int64_t &ns) {
    if (res >= 0) lo -= ((lo - res) % 8 + 8) % 8;
    int64_t n, m;
    sum_interval_size(hi - lo + 1, n, m);
    np += n;
    ns += m;
}
// columns with segments, listed in any order (one atomic per wavefront of kActiveSpan columns); the others get zero
// counts
constexpr int kActiveSpan = 512;
__global__ __launch_bounds__(kWG) void k_sum_active(SumWork sw) {
    const int lane = threadIdx.x & 63;
    const int64_t c0 = ((int64_t)blockIdx.x * (kWG / 64) + (threadIdx.x >> 6)) * kActiveSpan;
    uint64_t act[kActiveSpan / 64];
    uint32_t total = 0;
#pragma unroll
    for (int i = 0; i < kActiveSpan / 64; ++i) {
        const int64_t c = c0 + 64 * i + lane;
        bool has = false;
        if (c < sw.n_cols) {
            has = sw.col_seg_off[c + 1] > sw.col_seg_off[c];
            if (!has) {
                sw.piece_off[c] = 0;
                sw.s_off[c] = 0;
            }
        }
        act[i] = __ballot(has);
        total += (uint32_t)__builtin_popcountll(act[i]);
    }
    uint32_t base = 0;
    if (total && lane == 0) base = atomicAdd(sw.n_active, total);
    base = __shfl(base, 0);
#pragma unroll
    for (int i = 0; i < kActiveSpan / 64; ++i) {
        if ((act[i] >> lane) & 1ull)
            sw.active[base + __builtin_popcountll(act[i] & ((1ull << lane) - 1ull))] = (int32_t)(c0 + 64 * i + lane);
        base += (uint32_t)__builtin_popcountll(act[i]);
    }
}

__global__ __launch_bounds__(kWG) void k_sum_columns(int32_t align_res, const SegInfo *__restrict__ si, SumWork sw) {
    const int lane = threadIdx.x & 63;
    const uint64_t *__restrict__ in = sw.col_tmp;
    uint64_t *seg = sw.col_seg;
    const uint32_t n_act = *sw.n_active;
    const uint32_t waves = gridDim.x * (kWG / 64);
    for (uint32_t ia = blockIdx.x * (kWG / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); ia < n_act;
         ia += waves) {
        const int64_t cc = __builtin_amdgcn_readfirstlane(sw.active[ia]);
        const int64_t lb = sw.col_seg_off[cc], n = sw.col_seg_off[cc + 1] - lb;
        int32_t run_hi = 0, cur_lo = 0;                 // last tick of every entry so far; first tick of the open interval
        int64_t np = 0, ns = 0;                         // this lane's share of the column's counts
        // one 64-entry chunk of the sorted list: (first tick, last tick) of entry i0 + lane where `mine`
        auto chunk = [&](int64_t i0, bool mine, int32_t a0, int32_t end) {
            if (!mine) end = INT32_MIN;
            int32_t incl = end;                         // inclusive prefix maximum of the last ticks
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int32_t y = __shfl_up(incl, d);
                if (lane >= d) incl = max(incl, y);
            }
            int32_t excl = __shfl_up(incl, 1);
            if (lane == 0) excl = INT32_MIN;
            if (i0 > 0) excl = max(excl, run_hi);
            const bool st = mine && i0 + lane > 0 && (int64_t)a0 - excl - 1 > kSumGap;
            const uint64_t starts = __ballot(st);
            // the interval that ends before start lane s began at the previous start (or the open one)
            const uint64_t below = starts & ((1ull << lane) - 1ull);
            const int pl = below ? 63 - __builtin_clzll(below) : -1;
            const int32_t prev_lo = __shfl(a0, max(pl, 0));
            if (i0 == 0) cur_lo = __shfl(a0, 0);        // (shuffles in uniform control flow: every lane is a source)
            if (st) interval_count(pl >= 0 ? prev_lo : cur_lo, excl, align_res, np, ns);
            if (starts) cur_lo = __shfl(a0, 63 - __builtin_clzll(starts));
            run_hi = i0 == 0 ? __shfl(incl, 63) : max(run_hi, __shfl(incl, 63));
        };
        if (n <= 64) {
            // the lengths are loaded before the sort and travel with their keys to the lanes of their ranks
            const bool mine = lane < n;
            const uint64_t x = mine ? in[lb + lane] : ~0ull;
            const int32_t na = mine ? sw.segc[key_seg(x)].na : 0;
            int32_t rank = 0;
            for (int j = 0; j < (int)n; ++j) rank += lane_u64(x, j) < x;
            if (!mine) rank = lane;
            if (mine) seg[lb + rank] = x;
            const uint32_t xs_lo = (uint32_t)__builtin_amdgcn_ds_permute(rank * 4, (int)(uint32_t)x);
            const uint32_t xs_hi = (uint32_t)__builtin_amdgcn_ds_permute(rank * 4, (int)(uint32_t)(x >> 32));
            const int32_t nas = __builtin_amdgcn_ds_permute(rank * 4, na);
            const int32_t a0 = key_a0(((uint64_t)xs_hi << 32) | xs_lo);
            chunk(0, mine, a0, a0 + nas - 1);
        } else {
            for (int64_t i0 = 0; i0 < n; i0 += 64) {
                const bool mine = i0 + lane < n;
                const uint64_t x = mine ? in[lb + i0 + lane] : 0;
                int64_t rank = 0;
                for (int64_t j0 = 0; j0 < n; j0 += 64) {
                    const uint64_t y = j0 + lane < n ? in[lb + j0 + lane] : ~0ull;
                    const int jn = (int)min<int64_t>(64, n - j0);
                    for (int j = 0; j < jn; ++j) rank += lane_u64(y, j) < x;
                }
                if (mine) seg[lb + rank] = x;
            }
            // the sorted list before the wavefront reads it back
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            for (int64_t i0 = 0; i0 < n; i0 += 64) {
                const bool mine = i0 + lane < n;
                int32_t a0 = 0, end = 0;
                if (mine) {
                    const uint64_t x = seg[lb + i0 + lane];
                    a0 = key_a0(x);
                    end = a0 + sw.segc[key_seg(x)].na - 1;
                }
                chunk(i0, mine, a0, end);
            }
        }
        if (lane == 0) interval_count(cur_lo, run_hi, align_res, np, ns);     // the last interval
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            np += __shfl_xor(np, o);
            ns += __shfl_xor(ns, o);
        }
        if (lane == 0) {
            sw.piece_off[cc] = np;
            sw.s_off[cc] = ns;
        }
    }
}

void launch_sum_fill(const DevParams &P, const Work &w, const SumWork &sw, hipStream_t st) {
    if (w.n_seg > 0)
        k_sum_fill<<<(unsigned)((w.n_seg + kWG / 64 - 1) / (kWG / 64)), kWG, 0, st>>>(P, w.si, w.n_seg, sw);
    const int64_t span = (int64_t)(kWG / 64) * kActiveSpan;
    k_sum_active<<<(unsigned)((sw.n_cols + span - 1) / span), kWG, 0, st>>>(sw);
    k_sum_columns<<<256 * 16, kWG, 0, st>>>(sw.align_res, w.si, sw);   // persistent waves over the listed columns
}

// Wave-uniform copies of a 64-bit value held by lane l.
__device__ __forceinline__ int64_t uniform_i64(int64_t v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// per column: piece records, and the summed charge of each tick (Kahan over the column's segments in list order).
// Wavefronts take the columns with pieces from the active list, one column at a time; lane j sums tick
// lo + 64 m + j of the current interval over the interval's segments, the same additions per tick, in the same
// order, as a tick-by-tick scan.  For a list of at most kPieceStage segments, the lanes first stage each segment's
// first tick, length and cell base in this column in the wavefront's LDS slice, so the per-segment loops read them
// with one broadcast LDS read into scalar registers and only the (coalesced) cell loads go to memory; longer lists
// read each record in the loop.
constexpr int kPieceStage = 256;
struct SumRec {
    int32_t a0, na;
    int64_t base;                                       // cells index of tick 0 of the segment in this column
};
__global__ __launch_bounds__(kWG) void k_sum_pieces(DevParams P, const SegInfo *si, const float *cells, SumWork sw) {
    __shared__ SumRec stage_all[kWG / 64][kPieceStage];
    __shared__ int32_t rmax_all[kWG / 64][kPieceStage];
    const int lane = threadIdx.x & 63;
    SumRec *rs = stage_all[threadIdx.x >> 6];
    int32_t *rmax = rmax_all[threadIdx.x >> 6];       // last tick of entries 0 .. k (a running maximum)
    const int32_t res = sw.align_res;
    const uint32_t n_act = *sw.n_active;
    const uint32_t waves = gridDim.x * (kWG / 64);
    for (uint32_t ia = blockIdx.x * (kWG / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); ia < n_act;
         ia += waves) {
        const int64_t cc = __builtin_amdgcn_readfirstlane(sw.active[ia]);
        const int32_t e = (int32_t)(cc / ((int64_t)sw.CU * sw.CV));
        const int64_t r = cc - (int64_t)e * sw.CU * sw.CV;
        const int32_t u = sw.UL + (int32_t)(r / sw.CV), v = sw.VL + (int32_t)(r % sw.CV);
        const int64_t sb = sw.col_seg_off[cc], se = sw.col_seg_off[cc + 1], n = se - sb;
        int64_t pk = sw.piece_off[cc], so = sw.s_off[cc];
        const bool staged = n <= kPieceStage;
        // the previous column's reads of the slice are done before it is overwritten
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        uint64_t smask[kPieceStage / 64] = {};            // interval starts among the staged entries
        if (staged) {
            // records, and the interval starts by the rule k_sum_columns counts by (first tick more than kSumGap
            // beyond the running maximum of the earlier last ticks)
            int32_t carry = INT32_MIN;
#pragma unroll
            for (int w = 0; w < kPieceStage / 64; ++w) {
                if (64 * w >= n) break;
                const int64_t k = 64 * w + lane;
                const bool mine = k < n;
                int32_t a0 = 0, end = INT32_MIN;
                if (mine) {
                    const SumSeg g = sw.segc[key_seg(sw.col_seg[sb + k])];
                    a0 = g.a0;
                    end = g.a0 + g.na - 1;
                    rs[k] = SumRec{g.a0, g.na, g.cell_off + ((int64_t)(u - g.u0) * g.nv + (v - g.v0)) * g.na_pad - g.a0};
                }
                int32_t incl = end;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const int32_t y = __shfl_up(incl, d);
                    if (lane >= d) incl = max(incl, y);
                }
                incl = max(incl, carry);
                int32_t excl = __shfl_up(incl, 1);
                if (lane == 0) excl = carry;
                smask[w] = __ballot(mine && (k == 0 || (int64_t)a0 - excl - 1 > kSumGap));
                if (mine) rmax[k] = incl;
                carry = __shfl(incl, 63);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        // the interval starting at entry q of a staged list: its end entry qe (the next start) and last tick
        auto staged_interval = [&](int64_t q, int64_t &qe, int32_t &hi) {
            qe = n;
            for (int w = (int)((q + 1) >> 6); w < kPieceStage / 64 && 64 * w < n; ++w) {
                const uint64_t m = smask[w] & (((q + 1) >> 6) == w ? ~0ull << ((q + 1) & 63) : ~0ull);
                if (m) {
                    qe = 64 * w + __builtin_ctzll(m);
                    break;
                }
            }
            hi = __builtin_amdgcn_readfirstlane(rmax[qe - 1]);
        };
        auto from_lds = [&](int64_t k, int32_t &a0, int32_t &na, int64_t &base) {
            const SumRec x = rs[k];                         // the same address in every lane: a broadcast read
            a0 = __builtin_amdgcn_readfirstlane(x.a0);
            na = __builtin_amdgcn_readfirstlane(x.na);
            base = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)((uint64_t)x.base >> 32)) << 32) |
                             (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x.base));
        };
        auto from_global = [&](int64_t k, int32_t &a0, int32_t &na, int64_t &base) {
            const SumSeg g = sw.segc[key_seg(sw.col_seg[sb + k])];
            a0 = g.a0;
            na = g.na;
            base = g.cell_off + ((int64_t)(u - g.u0) * g.nv + (v - g.v0)) * g.na_pad - g.a0;
        };
        auto column = [&](auto seg_at, bool scanned) {
            for (int64_t q = 0; q < n;) {
                // the merged interval starting at list entry q (the rule k_sum_columns counts by)
                int32_t lo, hi, a0, na;
                int64_t base;
                seg_at(q, a0, na, base);
                lo = a0;
                hi = a0 + na - 1;
                int64_t qe = q + 1;
                if (scanned) {
                    staged_interval(q, qe, hi);
                } else {
                    for (; qe < n; ++qe) {
                        seg_at(qe, a0, na, base);
                        if (a0 - hi - 1 > kSumGap) break;
                        hi = max(hi, a0 + na - 1);
                    }
                }
                if (res >= 0) lo -= ((lo - res) % 8 + 8) % 8;
                const int32_t L = hi - lo + 1;
                int64_t np, Lpad;
                sum_interval_size(L, np, Lpad);
                float *S = sw.S + so;
                for (int32_t a0c = 0; a0c < Lpad; a0c += 64) {
                    const int32_t aa = lo + a0c + lane, ch = min(lo + a0c + 63, hi);
                    float sum = 0.0f, cmp = 0.0f;
                    // eight segments at a time: their cell loads are issued together, then added in list order
                    bool past = false;
                    for (int64_t k0 = q; k0 < qe && !past; k0 += 8) {
                        float val[8];
                        bool use[8];
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            use[i] = false;
                            val[i] = 0.0f;
                            if (k0 + i < qe && !past) {
                                seg_at(k0 + i, a0, na, base);
                                if (a0 > ch) past = true;           // sorted by first tick: no later one reaches
                                else if (aa >= a0 && aa <= a0 + na - 1 && aa <= hi) {
                                    use[i] = true;
                                    val[i] = cells[base + aa];
                                }
                            }
                        }
#pragma unroll
                        for (int i = 0; i < 8; ++i)
                            if (use[i]) {
                                const float y = val[i] - cmp;
                                const float t = sum + y;
                                cmp = (t - sum) - y;
                                sum = t;
                            }
                    }
                    if (a0c + lane < Lpad) S[a0c + lane] = sum - cmp;
                }
                for (int64_t k = lane; k < np; k += 64) {
                    SegInfo g = {};
                    g.u0 = u; g.nu = 1; g.v0 = v; g.nv = 1;
                    g.a0 = lo + (int32_t)k * kPieceTicks;
                    g.na = min(kPieceTicks, L - (int32_t)k * kPieceTicks);
                    g.na_pad = (g.na + kAC - 1) / kAC * kAC;
                    g.cell_off = so + k * kPieceTicks;
                    g.event = e;
                    g.n_pairs = 1;
                    if (sw.piece_lists) sw.piece[pk + k] = g;
                    sw.pdesc[pk + k] = PieceRef{g.a0, g.na, (uint32_t)(g.cell_off / kAC), 0};
                }
                pk += np;
                so += Lpad;
                q = qe;
            }
        };
        if (staged) column(from_lds, true);
        else column(from_global, false);
    }
}

void launch_sum_pieces(const DevParams &P, const Work &w, const SumWork &sw, hipStream_t st) {
    k_sum_pieces<<<256 * 16, kWG, 0, st>>>(P, w.si, w.cells, sw);   // persistent waves over the active columns
}

// per active pixel (one wavefront): number of column pieces in its table reach, then their ids and records in column
// order (row du, then column dv; pieces of a column in tick order).  The lanes take 64 consecutive columns at a time;
// a wavefront prefix sum of their piece counts gives each lane its place in the list.  A record is the piece's
// compact descriptor with the folded table column the pixel sees the column through, fold(du - bx) * by +
// fold(dv - by) for the column at offset (du, dv) of the pixel's reach.
// per active pixel: the number of column pieces in its reach (the columns of its +-bx x +-by sub-pixel window)
__global__ __launch_bounds__(kWG) void k_sum_lists_count(DevParams P, int64_t n_slots, const int32_t *slot_gp,
                                                         SumWork sw) {
    const int lane = threadIdx.x & 63;
    const int64_t slot = (int64_t)blockIdx.x * (kWG / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (slot >= n_slots) return;
    const int32_t gp = slot_gp[slot];
    const int32_t e = gp / P.npx, p = gp - e * P.npx;
    const int32_t ix = p % P.nx, iy = p / P.nx;
    const int32_t cu0 = ix * P.nsub + P.nsub / 2 - P.bx - sw.UL, cv0 = iy * P.nsub + P.nsub / 2 - P.by - sw.VL;
    const int64_t base = (int64_t)e * sw.CU * sw.CV;
    // piece_off is the exclusive prefix over the columns in row order: a row's 2 by columns of the reach count
    // piece_off[end] - piece_off[start]
    int64_t x = 0;
    for (int32_t du = lane; du < 2 * P.bx; du += 64) {
        const int64_t row = base + (int64_t)(cu0 + du) * sw.CV + cv0;
        x += sw.piece_off[row + 2 * P.by] - sw.piece_off[row];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (lane == 0) sw.list_off[slot] = x;
}

// per active pixel: its reach's column pieces as records, grouped by the folded table column (bin) the pixel sees
// them through and, within a bin, ascending in first tick (equal first ticks keep the mirror columns in the order
// du >= 0 before du < 0, then dv likewise).  Lane i merges the four tick-sorted piece lists of bin b0 + i.
__global__ __launch_bounds__(kWG) void k_sum_lists_fill(DevParams P, int64_t n_slots, const int32_t *slot_gp,
                                                        SumWork sw) {
    const int lane = threadIdx.x & 63;
    const int64_t slot = (int64_t)blockIdx.x * (kWG / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (slot >= n_slots) return;
    const int32_t gp = slot_gp[slot];
    const int32_t e = gp / P.npx, p = gp - e * P.npx;
    const int32_t ix = p % P.nx, iy = p / P.nx;
    const int32_t cu0 = ix * P.nsub + P.nsub / 2 - sw.UL, cv0 = iy * P.nsub + P.nsub / 2 - sw.VL;   // centre column
    const int64_t base = (int64_t)e * sw.CU * sw.CV;
    const int32_t nbin = P.bx * P.by;
    int64_t pos = sw.list_off[slot];
    for (int32_t b0 = 0; b0 < nbin; b0 += 64) {
        const int32_t b = b0 + lane;
        int64_t h[4] = {0, 0, 0, 0}, he[4] = {0, 0, 0, 0};
        int64_t x = 0;
        if (b < nbin) {
            const int32_t fu = b / P.by, fv = b - fu * P.by;
#pragma unroll
            for (int m = 0; m < 4; ++m) {                // the four columns whose offsets fold to (fu, fv)
                const int32_t du = (m & 1) ? -fu - 1 : fu, dv = (m & 2) ? -fv - 1 : fv;
                const int64_t col = base + (int64_t)(cu0 + du) * sw.CV + (cv0 + dv);
                h[m] = sw.piece_off[col];
                he[m] = sw.piece_off[col + 1];
                x += he[m] - h[m];
            }
        }
        int64_t incl = x;                               // inclusive prefix of the lanes' record counts
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t y = __shfl_up(incl, d);
            if (lane >= d) incl += y;
        }
        if (x) {
            int32_t ha[4];                              // first tick at each list's head (INT32_MAX when empty)
#pragma unroll
            for (int m = 0; m < 4; ++m) ha[m] = h[m] < he[m] ? sw.pdesc[h[m]].a0 : INT32_MAX;
            for (int64_t q = pos + incl - x; q < pos + incl; ++q) {
                int m = 0;
#pragma unroll
                for (int j = 1; j < 4; ++j) m = ha[j] < (m == 0 ? ha[0] : m == 1 ? ha[1] : ha[2]) ? j : m;
                int64_t k = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (j == m) {
                        k = h[j]++;
                        ha[j] = h[j] < he[j] ? sw.pdesc[h[j]].a0 : INT32_MAX;
                    }
                if (sw.piece_lists) sw.list[q] = (int32_t)k;
                PieceRef r = sw.pdesc[k];
                r.bin = b;
                sw.rec[q] = r;
            }
        }
        pos += __shfl(incl, 63);
    }
}

void launch_sum_lists_count(const DevParams &P, const Work &w, const SumWork &sw, int64_t n_slots, hipStream_t st) {
    if (n_slots > 0)
        k_sum_lists_count<<<(unsigned)((n_slots + kWG / 64 - 1) / (kWG / 64)), kWG, 0, st>>>(P, n_slots, w.slot_gp, sw);
}
void launch_sum_lists_fill(const DevParams &P, const Work &w, const SumWork &sw, int64_t n_slots, int64_t n_list,
                           hipStream_t st) {
    if (n_slots > 0)
        k_sum_lists_fill<<<(unsigned)((n_slots + kWG / 64 - 1) / (kWG / 64)), kWG, 0, st>>>(P, n_slots, w.slot_gp, sw);
    (void)n_list;
}

// Mirror merge.  A pixel convolves every record of one folded table column with the same table column, so a run of
// its list's records with the same bin whose tick spans overlap or lie at most kMergeGap ticks apart is one record
// whose charge is the members' sum, taken in list order (a member's charge sits at its first tick's offset from the
// union's first tick).  Runs are cut at every 64th record of the pixel's
// list (the lanes of one pass), and a run whose union would exceed kPieceMax ticks is not merged; a run of one record
// stays as it is.  Count pass: records and merged-charge floats per pixel; fill pass: the merged records (in list
// order) and their charges.  One wavefront per pixel; the runs of 64 records are found with segmented lane scans.
constexpr int32_t kMergeGap = 8;

// Inclusive segmented scans over the wavefront (a segment starts at a lane whose flag is set).
__device__ __forceinline__ int32_t seg_scan_max(int32_t v, bool start) {
    const int lane = lane_id();
    int f = start;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t y = __shfl_up(v, d);
        const int g = __shfl_up(f, d);
        if (lane >= d && !f) {
            v = max(v, y);
            f |= g;
        }
    }
    return v;
}
__device__ __forceinline__ int32_t seg_scan_min(int32_t v, bool start) {
    const int lane = lane_id();
    int f = start;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t y = __shfl_up(v, d);
        const int g = __shfl_up(f, d);
        if (lane >= d && !f) {
            v = min(v, y);
            f |= g;
        }
    }
    return v;
}
template <bool FILL>
__global__ __launch_bounds__(kWG) void k_sum_merge(int64_t n_slots, SumWork sw) {
    const int lane = threadIdx.x & 63;
    const int64_t slot = (int64_t)blockIdx.x * (kWG / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (slot >= n_slots) return;
    const int64_t pb = sw.list_off[slot], pe = sw.list_off[slot + 1];
    int64_t ng = FILL ? sw.mlist_off[slot] : 0, nm = FILL ? sw.m_off[slot] : 0;
    for (int64_t c0 = pb; c0 < pe; c0 += 64) {
        const int32_t n = (int32_t)min<int64_t>(64, pe - c0);
        const bool in = lane < n;
        PieceRef r{0, 0, 0, 0};
        if (in) r = sw.rec[c0 + lane];
        const int32_t end = r.a0 + r.na - 1;
        // runs: a new bin, or a first tick beyond the bin's spans so far (first ticks ascend within a bin) + the gap
        const bool fb = lane == 0 || r.bin != __shfl_up(r.bin, 1);
        const int32_t mb = seg_scan_max(end, fb);
        const int32_t mprev = __shfl_up(mb, 1);
        bool st = fb || r.a0 > mprev + 1 + kMergeGap;
        const int32_t ghi = seg_scan_max(end, st);       // the run's last tick so far
        const int32_t glo = seg_scan_min(r.a0, st);      // its first tick
        // each record's natural run ends before the next run start; the verdict on the run's span is read there
        const uint64_t nat = __ballot(in && st);
        const uint64_t nat_after = lane == 63 ? 0ull : nat >> (lane + 1);
        const int32_t run_end = nat_after ? lane + __builtin_ctzll(nat_after) : n - 1;
        const bool ok = __shfl((int)(ghi - glo + 1 <= kPieceMax), max(min(run_end, 63), 0)) != 0;
        st = in && (st || !ok);                         // runs over kPieceMax ticks stay single records
        const uint64_t starts = __ballot(st);
        const uint64_t after = lane == 63 ? 0ull : starts >> (lane + 1);
        const int32_t nxt = after ? lane + 1 + __builtin_ctzll(after) : n;
        const int32_t rhi = __shfl(ghi, max(nxt - 1, 0));
        const bool multi = st && nxt - lane > 1;
        const int32_t L = multi ? rhi - r.a0 + 1 : r.na;
        const int32_t Lp = multi ? (L + kAC - 1) / kAC * kAC : 0;
        int64_t incl = Lp;                              // inclusive prefix of the merged-charge floats
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t y = __shfl_up(incl, d);
            if (lane >= d) incl += y;
        }
        if (FILL) {
            const int64_t moff = nm + incl - Lp;
            if (st) {
                const int64_t g = ng + __builtin_popcountll(starts & ((1ull << lane) - 1ull));
                sw.mrec[g] = multi ? PieceRef{r.a0, L, sw.nS8 + (uint32_t)(moff / kAC), r.bin} : r;
            }
            uint64_t mm = __ballot(multi);
            while (mm) {                                // each merged run: its charge, lanes over its ticks
                const int i = __builtin_ctzll(mm);
                mm &= mm - 1ull;
                const int32_t lo = __builtin_amdgcn_readlane(r.a0, i);
                const int32_t ke = __builtin_amdgcn_readlane(nxt, i);
                const int32_t lp = __builtin_amdgcn_readlane(Lp, i);
                const int64_t off = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(moff >> 32), i) << 32) |
                                              (uint32_t)__builtin_amdgcn_readlane((int)moff, i));
                for (int32_t t0 = 0; t0 < lp; t0 += 64) {
                    float v = 0.0f;
                    for (int32_t k0 = i; k0 < ke; k0 += 4) {  // members in list order, four loads in flight
                        float x[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            x[q] = 0.0f;
                            const int32_t k = min(k0 + q, 63);
                            const int32_t ma = __builtin_amdgcn_readlane(r.a0, k);
                            const int32_t mn = __builtin_amdgcn_readlane(r.na, k);
                            const uint32_t mc = (uint32_t)__builtin_amdgcn_readlane((int)r.cell8, k);
                            const int32_t o = lo + t0 + lane - ma;
                            if (k0 + q < ke && o >= 0 && o < mn) x[q] = sw.S[(int64_t)mc * kAC + o];
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q) v += x[q];  // adding an exact zero leaves v unchanged
                    }
                    if (t0 + lane < lp) sw.Sm[off + t0 + lane] = v;
                }
            }
        }
        ng += __builtin_popcountll(starts);
        nm += __shfl(incl, 63);
    }
    if (!FILL && lane == 0) {
        sw.mlist_off[slot] = ng;
        sw.m_off[slot] = nm;
    }
}

void launch_sum_merge(const SumWork &sw, int64_t n_slots, bool fill, hipStream_t st) {
    if (n_slots <= 0) return;
    const unsigned g = (unsigned)((n_slots + kWG / 64 - 1) / (kWG / 64));
    if (fill) k_sum_merge<true><<<g, kWG, 0, st>>>(n_slots, sw);
    else k_sum_merge<false><<<g, kWG, 0, st>>>(n_slots, sw);
}

// Summed induction, one wavefront per work unit (active pixel, tile of kTileTicks ticks): lane t owns ticks
// t0 + 8t .. +7 of the tile, and the wavefront streams every column piece of the pixel's list whose tick window
// [a0 - T_R + 1, a0 + na - 1] meets the tile through the four-block register ring, three blocks ahead and into the
// next piece (pieces start at the aligning residue, so every lane's table offset is a multiple of 8 and the loads
// are aligned 16-byte loads).  The pieces come as 16-byte records (first tick, length, charge offset, folded table
// column), so the walk needs no dependent loads.  Lanes whose ticks lie outside a piece's window read the table's
// zero padding, so they add exact zeros.  The products are added to the lane's running sums with Kahan
// compensation after every 4 pieces (pieces in list order: deterministic and batch-invariant).  Wavefronts take
// units from a counter and never synchronise with each other; the first tile of a pixel also accounts the charge
// that its pieces induce outside the window.
// A record's summed charge: in the column pieces' buffer, or in the merged records' one.
__device__ __forceinline__ const float *cell_ptr(const float *S, const float *Sm, uint32_t nS8, uint32_t cell8) {
    return cell8 < nS8 ? S + (int64_t)cell8 * kAC : Sm + (int64_t)(cell8 - nS8) * kAC;
}

constexpr int32_t kSumKahanEvery = 4;   // pieces summed in FP32 registers between compensated additions

template <bool SHIFT>
__global__ __launch_bounds__(kWG) void k_induce_summed(DevParams P, const SegInfo *__restrict__ piece,
                                                       const float *__restrict__ S, const float *__restrict__ Sm,
                                                       uint32_t nS8, const float *__restrict__ Rpad,
                                                       const double *__restrict__ prefix,
                                                       const int64_t *__restrict__ list_off,
                                                       const int32_t *__restrict__ list,
                                                       const PieceRef *__restrict__ rec,
                                                       const int32_t *__restrict__ order,
                                                       const int32_t *__restrict__ slot_gp, float *__restrict__ wave,
                                                       DevHeader *H, double *report) {
    const int lane = threadIdx.x & 63;
    const int32_t NT = P.nticks, TR = P.t_r;
    const int32_t n_tiles = (NT + kTileTicks - 1) / kTileTicks;
    const int64_t n_units = H->n_slots * n_tiles;
    for (;;) {
        uint32_t got = 0;
        if (lane == 0) got = atomicAdd(&H->work[2], 1u);
        const int64_t unit = (int64_t)__builtin_amdgcn_readfirstlane(__shfl(got, 0));
        if (unit >= n_units) break;
        const int64_t ui = unit / n_tiles;
        const int64_t slot = order ? order[ui] : ui;                    // largest-first when an order is given
        const int32_t t0 = (int32_t)(unit - ui * n_tiles) * kTileTicks, t1 = t0 + kTileTicks - 1;
        const int32_t gp = slot_gp[slot];
        const int32_t e = gp / P.npx, p = gp - e * P.npx;
        const int32_t uc = (p % P.nx) * P.nsub + P.nsub / 2, vc = (p / P.nx) * P.nsub + P.nsub / 2;
        const int32_t nb = t0 + 8 * lane;
        const int64_t pb = list_off[slot], pe = list_off[slot + 1];
        float acc[8], sum[8], cmp[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) { acc[r] = 0.0f; sum[r] = 0.0f; cmp[r] = 0.0f; }
        auto meets = [&](int64_t k) {
            const SegInfo &g = piece[list[k]];
            return g.a0 + g.na - 1 >= t0 && g.a0 - (TR - 1) <= t1;
        };
        auto colof = [&](int64_t k, const float *&col, const float *&cc, int32_t &nblk) {
            const SegInfo &g = piece[list[k]];
            col = Rpad + (int64_t)(fold(g.u0 - uc) * P.by + fold(g.v0 - vc)) * P.col_len + (nb - g.a0 + TR - 1 + kPad);
            cc = S + g.cell_off;
            nblk = g.na_pad / kAC;
        };
        if constexpr (!SHIFT) {                         // aligned ping-pong per piece, Kahan after every 4 pieces
            auto kahan = [&] {
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const float y = acc[r] - cmp[r];
                    const float t = sum[r] + y;
                    cmp[r] = (t - sum[r]) - y;
                    sum[r] = t;
                    acc[r] = 0.0f;
                }
            };
            // the pixel's pieces that meet the tile, in list order, streamed through the four-block register ring
            // (three blocks ahead, the next piece's first blocks loaded while the current one runs)
            auto skip = [&](int64_t q) {
                while (q < pe) {
                    const PieceRef r = rec[q];
                    if (r.a0 + r.na - 1 >= t0 && r.a0 - (TR - 1) <= t1) break;
                    ++q;
                }
                return q;
            };
            int32_t pending = 0;
            int64_t q = skip(pb);
            if (q < pe) {
                auto colp = [&](const PieceRef &r) {
                    return Rpad + (int64_t)r.bin * P.col_len + (nb - r.a0 + TR - 1 + kPad);
                };
                const PieceRef r0 = rec[q];
                auto adv = [&](const float *&ncol, const float *&ncc, int32_t &nn) {
                    q = skip(q + 1);
                    if (q >= pe) return false;
                    const PieceRef r = rec[q];
                    ncol = colp(r);
                    ncc = cell_ptr(S, Sm, nS8, r.cell8);
                    nn = (r.na + kAC - 1) / kAC;
                    return true;
                };
                auto done = [&] {
                    if (++pending == kSumKahanEvery) {
                        kahan();
                        pending = 0;
                    }
                };
                column_stream<false, true>(colp(r0), cell_ptr(S, Sm, nS8, r0.cell8), (r0.na + kAC - 1) / kAC, adv,
                                           done, acc);
            }
            if (pending) kahan();
        } else {
            int64_t q = pb;
            while (q < pe && !meets(q)) ++q;
            if (q < pe) {
                const float *col, *cc;
                int32_t nblk;
                colof(q, col, cc, nblk);
                auto adv = [&](const float *&ncol, const float *&ncc, int32_t &nn) {
                    do { ++q; } while (q < pe && !meets(q));
                    if (q >= pe) return false;
                    colof(q, ncol, ncc, nn);
                    return true;
                };
                auto done = [&] {
#pragma unroll
                    for (int r = 0; r < 8; ++r) {
                        const float y = acc[r] - cmp[r];
                        const float t = sum[r] + y;
                        cmp[r] = (t - sum[r]) - y;
                        sum[r] = t;
                        acc[r] = 0.0f;
                    }
                };
                column_stream<SHIFT, false>(col, cc, nblk, adv, done, acc);
            }
        }
        float *wrow = wave + slot * NT;
#pragma unroll
        for (int r = 0; r < 8; ++r)
            if (nb + r < NT) wrow[nb + r] = sum[r] - cmp[r];
        if (t0 == 0) {                                  // charge induced outside [0, NT) by the pixel's pieces
            double clip = 0.0;
            for (int64_t k = pb + lane; k < pe; k += 64) {
                const PieceRef g = rec[k];
                const int32_t wlo = g.a0 - (TR - 1), whi = g.a0 + g.na - 1;
                if (wlo >= 0 && whi < NT) continue;
                const double *pf = prefix + (int64_t)g.bin * (TR + 1);
                const float *cv = cell_ptr(S, Sm, nS8, g.cell8);
                for (int32_t a = 0; a < g.na; ++a) {
                    const int32_t aa = g.a0 + a;
                    const int32_t klo = min(max(TR - 1 - aa, 0), TR), khi = min(max(NT + TR - 1 - aa, 0), TR);
                    const double dropped = klo >= khi ? pf[TR] : pf[klo] + (pf[TR] - pf[khi]);
                    clip += (double)cv[a] * dropped;
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) clip += __shfl_xor(clip, o);
            if (lane == 0 && clip != 0.0) atomicAdd(&report[(int64_t)e * 5 + 3], clip);
        }
    }
}

// Summed induction in 256-tick work units (active pixel, tile of kTile4 ticks), one wavefront each: lane t owns
// ticks t0 + 4t .. +3.  The pixel's records are scanned 64 at a time (a ballot of those whose tick window
// [a0 - T_R + 1, a0 + na - 1] meets the tile); for each, the wavefront stages the table values the tile needs
// (index t0 - a0 - nap + 1 .. t0 - a0 + 255 of the column, relative to its lag-0 entry) in its LDS slice with aligned
// 16-byte copies, then streams the record's 8-tick charge blocks (uniform loads) against a 12-value window that moves
// down 8 values per block (two aligned LDS reads per block).  Lanes whose ticks lie outside the record's window meet
// the table's zero padding.  Products go to the lane's running sums with Kahan compensation after every 4 records
// (records in list order: deterministic and batch-invariant).  The first tile of a pixel also accounts the charge
// its records induce outside the readout.  Charge intervals start at any tick: the staged copy is loaded from the
// 16-byte aligned column entry at or below its first value and written to LDS shifted down by the difference.
constexpr int32_t kTile4 = 256;                         // ticks of one work unit: 64 lanes x 4
constexpr int32_t kStage4 = kTile4 + kPieceMax + 8;     // staged table values per record and unit (at most)

// Block of 4 ticks x 8 charge ticks: tick r of the lane against charge tick q uses window value r - q + 7.
__device__ __forceinline__ void block4(const float (&w)[12], const float (&c)[kAC], float (&acc)[4]) {
#pragma unroll
    for (int q = 0; q < kAC; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = fmaf(c[q], w[r - q + 7], acc[r]);
}
__device__ __forceinline__ void window4(const float *p, float (&w)[12]) {
    const float4 x = *(const float4 *)p, y = *(const float4 *)(p + 4), z = *(const float4 *)(p + 8);
    w[0] = x.x; w[1] = x.y; w[2] = x.z; w[3] = x.w; w[4] = y.x; w[5] = y.y; w[6] = y.z; w[7] = y.w;
    w[8] = z.x; w[9] = z.y; w[10] = z.z; w[11] = z.w;
}

__global__ __launch_bounds__(kWG) void k_induce_summed4(DevParams P, const float *__restrict__ S,
                                                        const float *__restrict__ Sm, uint32_t nS8,
                                                        const float *__restrict__ Rpad,
                                                        const double *__restrict__ prefix,
                                                        const int64_t *__restrict__ list_off,
                                                        const PieceRef *__restrict__ rec,
                                                        const int32_t *__restrict__ order,
                                                        const int32_t *__restrict__ slot_gp, float *__restrict__ wave,
                                                        DevHeader *H, double *report) {
    __shared__ __align__(16) float stage_all[kWG / 64][4 + kStage4];
    const int lane = threadIdx.x & 63;
    float *stage = stage_all[threadIdx.x >> 6] + 4;     // 4 head floats take the unneeded values of a shifted copy
    const int32_t NT = P.nticks, TR = P.t_r;
    const int32_t n_tiles = (NT + kTile4 - 1) / kTile4;
    const int64_t n_units = H->n_slots * n_tiles;
    for (;;) {
        uint32_t got = 0;
        if (lane == 0) got = atomicAdd(&H->work[2], 1u);
        const int64_t unit = (int64_t)__builtin_amdgcn_readfirstlane(__shfl(got, 0));
        if (unit >= n_units) break;
        const int64_t ui = unit / n_tiles;
        const int64_t slot = order ? order[ui] : ui;                    // largest-first when an order is given
        const int32_t t0 = (int32_t)(unit - ui * n_tiles) * kTile4, t1 = t0 + kTile4 - 1;
        const int32_t gp = slot_gp[slot];
        const int32_t e = gp / P.npx;
        const int64_t pb = list_off[slot], pe = list_off[slot + 1];
        float acc[4], sum[4], cmp[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) { acc[r] = 0.0f; sum[r] = 0.0f; cmp[r] = 0.0f; }
        int32_t pending = 0;
        for (int64_t c0 = pb; c0 < pe; c0 += 64) {
            PieceRef rl{0, 0, 0, 0};
            const bool in = c0 + lane < pe;
            if (in) rl = rec[c0 + lane];
            uint64_t mask = __ballot(in && rl.a0 + rl.na - 1 >= t0 && rl.a0 - (TR - 1) <= t1);
            if (!mask) continue;
            // record i of the chunk: its fields, and the lane's two staged float4s of it, loaded ahead
            int32_t a0 = 0, nblk = 0, n4 = 0, dl = 0;
            uint32_t c8 = 0;
            float4 g0 = {0, 0, 0, 0}, g1 = {0, 0, 0, 0};
            auto fetch = [&](int i) {
                a0 = __builtin_amdgcn_readlane(rl.a0, i);
                const int32_t na = __builtin_amdgcn_readlane(rl.na, i);
                const int32_t bin = __builtin_amdgcn_readlane(rl.bin, i);
                c8 = (uint32_t)__builtin_amdgcn_readlane((int)rl.cell8, i);
                nblk = (na + kAC - 1) / kAC;
                // the values staged are column entries idx0 .. idx0 + 255 + 8 nblk; they are loaded from the
                // 16-byte aligned entry idx0 - dl below (table columns start 32-byte aligned)
                const int32_t idx0 = t0 - a0 - nblk * kAC + TR + kPad;
                dl = idx0 & 3;
                n4 = (kTile4 + nblk * kAC + dl + 3) / 4;
                const float *src = Rpad + (int64_t)bin * P.col_len + (idx0 - dl);
                g0 = *(const float4 *)(src + 4 * lane);
                if (lane + 64 < n4) g1 = *(const float4 *)(src + 4 * (lane + 64));
            };
            while (mask) {
                const int i = __builtin_ctzll(mask);
                mask &= mask - 1ull;
                fetch(i);
                // the previous record's window reads are done before the slice is overwritten
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (dl == 0) {
                    *(float4 *)(stage + 4 * lane) = g0;
                    if (lane + 64 < n4) *(float4 *)(stage + 4 * (lane + 64)) = g1;
                } else {                                // dl entries down: lane 0's first ones land in the head
                    float *d0 = stage + 4 * lane - dl;
                    d0[0] = g0.x; d0[1] = g0.y; d0[2] = g0.z; d0[3] = g0.w;
                    if (lane + 64 < n4) {
                        float *d1 = d0 + 256;
                        d1[0] = g1.x; d1[1] = g1.y; d1[2] = g1.z; d1[3] = g1.w;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const int32_t nb_cur = nblk;
                cfloat_ptr cc = uniform_cptr(cell_ptr(S, Sm, nS8, c8));
                // 8-tick charge blocks against the 12-value window that moves down 8 per block (the latency of the
                // window and charge loads is covered by the other wavefronts of the SIMD)
                int32_t wb = 4 * lane + nb_cur * kAC - 8;
                for (int32_t j = 0; j < nb_cur; ++j, wb -= 8) {
                    float W[12], cv[kAC];
                    window4(stage + wb, W);
#pragma unroll
                    for (int q = 0; q < kAC; ++q) cv[q] = cc[kAC * j + q];
                    block4(W, cv, acc);
                }
                if (++pending == kSumKahanEvery) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float y = acc[r] - cmp[r];
                        const float t = sum[r] + y;
                        cmp[r] = (t - sum[r]) - y;
                        sum[r] = t;
                        acc[r] = 0.0f;
                    }
                    pending = 0;
                }
            }
        }
        if (pending) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float y = acc[r] - cmp[r];
                const float t = sum[r] + y;
                cmp[r] = (t - sum[r]) - y;
                sum[r] = t;
            }
        }
        float *wrow = wave + slot * NT;
        const int32_t nb = t0 + 4 * lane;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (nb + r < NT) wrow[nb + r] = sum[r] - cmp[r];
        if (t0 == 0) {                                  // charge induced outside [0, NT) by the pixel's records
            double clip = 0.0;
            for (int64_t k = pb + lane; k < pe; k += 64) {
                const PieceRef g = rec[k];
                const int32_t wlo = g.a0 - (TR - 1), whi = g.a0 + g.na - 1;
                if (wlo >= 0 && whi < NT) continue;
                const double *pf = prefix + (int64_t)g.bin * (TR + 1);
                const float *cv = cell_ptr(S, Sm, nS8, g.cell8);
                for (int32_t a = 0; a < g.na; ++a) {
                    const int32_t aa = g.a0 + a;
                    const int32_t klo = min(max(TR - 1 - aa, 0), TR), khi = min(max(NT + TR - 1 - aa, 0), TR);
                    const double dropped = klo >= khi ? pf[TR] : pf[klo] + (pf[TR] - pf[khi]);
                    clip += (double)cv[a] * dropped;
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) clip += __shfl_xor(clip, o);
            if (lane == 0 && clip != 0.0) atomicAdd(&report[(int64_t)e * 5 + 3], clip);
        }
    }
}

bool summed_tile256(int32_t rt, bool shift) { return rt == 0 && !shift; }
int32_t summed_align_res(const DevParams &P, int32_t rt, bool shift) {
    if (summed_tile256(rt, shift)) return -1;          // its staging copy realigns the table values itself
    return ((P.t_r - 1 + kPad) % 8 + 8) % 8;
}

// Largest-first order of the pixels for the summed induction (the same log-bucketed order as the per-pair kernel's;
// all tiles of a pixel stay together): work of a pixel = the cell-tick blocks of its pieces.
__global__ __launch_bounds__(kWG) void k_slot_work_summed(const PieceRef *__restrict__ rec,
                                                          const int64_t *__restrict__ list_off, int64_t n_slots,
                                                          int32_t *__restrict__ bucket, int32_t *__restrict__ hist) {
    const int lane = threadIdx.x & 63;                  // one wavefront per pixel, lanes over its records
    const int64_t slot = (int64_t)blockIdx.x * (kWG / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (slot >= n_slots) return;
    int64_t blocks = 0;                                 // an integer sum: the same in any order
    for (int64_t q = list_off[slot] + lane; q < list_off[slot + 1]; q += 64) blocks += (rec[q].na + kAC - 1) / kAC;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) blocks += __shfl_xor(blocks, o);
    if (lane == 0) {
        const double work = (double)blocks;
        const int32_t lg = work >= 1.0 ? (int32_t)(16.0 * log2(work)) : 0;
        const int32_t b = kOrderBuckets - 1 - min(lg, kOrderBuckets - 1);
        bucket[slot] = b;
        atomicAdd(&hist[b], 1);
    }
}

const int32_t *launch_summed_order(const Work &w, const SumWork &sw, int64_t n_slots, int32_t rt, bool shift,
                                   hipStream_t st) {
    if ((rt != 0 && rt != 8) || n_slots <= 0 || !w.order || shift) return nullptr;
    int32_t *ord = w.order, *bucket = ord + n_slots, *hist = bucket + n_slots, *cursor = hist + kOrderBuckets;
    launch_zero(hist, (int64_t)sizeof(int32_t) * kOrderBuckets, st);
    const unsigned gs = (unsigned)((n_slots + kWG - 1) / kWG);
    k_slot_work_summed<<<(unsigned)((n_slots + kWG / 64 - 1) / (kWG / 64)), kWG, 0, st>>>(sw.mrec, sw.mlist_off, n_slots,
                                                                                         bucket, hist);
    k_order_offsets<<<1, kWG, 0, st>>>(hist, cursor);
    k_order_scatter<<<gs, kWG, 0, st>>>(bucket, n_slots, cursor, ord);
    return ord;
}

void launch_induce_summed(const DevParams &P, const Work &w, const SumWork &sw, const Table &T, float *wave,
                          int64_t n_slots, int32_t rt, bool shift, const int32_t *order, hipStream_t st) {
    if (rt != 0 && rt != 8) {                           // the per-pair kernel on the summed pieces (tuning option)
        Work ws = w;
        ws.si = sw.piece;
        ws.cells = sw.S;
        ws.slot_off = sw.list_off;
        ws.pairs = sw.list;
        launch_induce(P, ws, T, wave, 0, n_slots, rt, false, st);
        return;
    }
    if (n_slots <= 0) return;
    if (summed_tile256(rt, shift)) {
        const int64_t units = n_slots * ((P.nticks + kTile4 - 1) / kTile4);
        const int64_t g = std::min<int64_t>((units + kWG / 64 - 1) / (kWG / 64), 256 * 8);
        k_induce_summed4<<<(unsigned)g, kWG, 0, st>>>(P, sw.S, sw.Sm, sw.nS8, T.Rpad, T.prefix, sw.mlist_off, sw.mrec,
                                                      order, w.slot_gp, wave, w.hdr, w.report);
        return;
    }
    const int64_t units = n_slots * ((P.nticks + kTileTicks - 1) / kTileTicks);
    const int64_t g = std::min<int64_t>((units + kWG / 64 - 1) / (kWG / 64), 256 * 8);
    if (shift)                                          // per piece (the list and the unmerged records)
        k_induce_summed<true><<<(unsigned)g, kWG, 0, st>>>(P, sw.piece, sw.S, sw.Sm, sw.nS8, T.Rpad, T.prefix,
                                                           sw.list_off, sw.list, sw.rec, order, w.slot_gp, wave,
                                                           w.hdr, w.report);
    else                                                // the merged records
        k_induce_summed<false><<<(unsigned)g, kWG, 0, st>>>(P, sw.piece, sw.S, sw.Sm, sw.nS8, T.Rpad, T.prefix,
                                                            sw.mlist_off, sw.list, sw.mrec, order, w.slot_gp, wave,
                                                            w.hdr, w.report);
}

// ================================================================================================= electronics
// Front-end electronics (Sec. 3.4), one wavefront per active pixel.  The per-tick rule: Q += I[n]; when no sample
// is pending and n >= ready, a crossing happens if Q + discriminator noise >= threshold; the sample is taken at
// max(n + hold, last + spacing) with uncorrelated noise added; ADC = clamp(floor(Q_s / q_lsb) + pedestal); the
// integrator restarts from the reset noise after the sample tick; a periodic reset applies before a tick's charge
// when no sample is pending.  The discriminator draw is skipped exactly when Q + |g|max * sigma_disc cannot reach
// the threshold.
//
// The walk goes in 64-tick chunks: the 64 lanes load a chunk at once, the charge and its absolute values since the
// segment start (the chunk start or the last reset) are prefix-summed across the lanes, and the events of the chunk
// (crossings, samples, resets) are found by ballots and handled in tick order; a lane's integrated charge is the
// value carried into the segment plus its prefix sum.  The carried value is a Kahan pair; a prefix sum over one
// segment of at most 64 ticks adds at most six roundings of its absolute sum, well inside the decision margin's
// relative term.  (One thread per pixel walking the ticks in order was 4.4x slower: too few wavefronts, and a
// dependent load per tick.)
__device__ __forceinline__ float lane_value(float v, int32_t l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int32_t, v), l));
}

__global__ __launch_bounds__(kWG) void k_electronics(DevParams P, const float *__restrict__ wave,
                                                     const int32_t *__restrict__ slot_gp,
                                                     const uint64_t *__restrict__ ev_ids, int32_t n_ev,
                                                     const uint8_t *__restrict__ disabled, int64_t n_slots_arg,
                                                     int32_t *pk_tick, uint16_t *pk_adc, uint8_t *pk_flag,
                                                     int64_t *pk_cnt, DevHeader *H, double *report,
                                                     int64_t *ev_cnt) {
    const int64_t n_slots = n_slots_arg >= 0 ? n_slots_arg : H->n_slots;
    const int32_t NT = P.nticks, RP = P.reset_period;
    const int lane = lane_id();
    constexpr int kWaves = kWG / 64;
    const int32_t wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int64_t slot = (int64_t)blockIdx.x * kWaves + wv; slot < n_slots; slot += (int64_t)gridDim.x * kWaves) {
        const int32_t gp = __builtin_amdgcn_readfirstlane(slot_gp[slot]);
        if (!(gp >= 0 && gp < n_ev * P.npx)) {                   // ids outside the event grids are skipped
            if (lane == 0) pk_cnt[slot] = 0;
            continue;
        }
        const int32_t e = gp / P.npx;
        const uint32_t pid = (uint32_t)(gp - e * P.npx);
        const bool off = disabled && disabled[pid];                   // disabled channel: no packets
        const uint64_t ev = ev_ids[e];
        const float *w = wave + slot * NT;
        const float reset0 = P.sig_reset > 0.0f ? P.sig_reset * noise_normal(P, pid, kTickInitial, ev, STREAM_RESET)
                                                : 0.0f;
        float Qb = reset0, Qbc = 0.0f, Ab = 0.0f;                     // carried charge (Kahan pair) and |charge|
        bool pending = false, uncertain = false, done = off;
        int32_t ns = 0, ready = 0, last = -(1 << 28), cnt = 0, dropped = 0, over = 0;
        const int64_t obase = slot * P.max_packets;
        double rs = 0.0;
        for (int32_t n0 = 0; n0 < NT; n0 += 64) {
            const int32_t n = n0 + lane;
            const float x = n < NT ? w[n] : 0.0f;
            rs += (double)x;
            if (done) continue;
            float sx, sa;                                             // prefix sums over lanes s..lane
            auto scan = [&](int32_t s) {
                sx = lane >= s ? x : 0.0f;
                sa = fabsf(sx);
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const float yx = __shfl_up(sx, d), ya = __shfl_up(sa, d);
                    if (lane >= d) { sx += yx; sa += ya; }
                }
            };
            auto restart = [&](uint32_t tick) {                       // integrator reset
                Qb = P.sig_reset > 0.0f ? P.sig_reset * noise_normal(P, pid, tick, ev, STREAM_RESET) : 0.0f;
                Qbc = 0.0f;
                Ab = 0.0f;
            };
            scan(0);
            const int32_t jn = min(64, NT - n0);
            int32_t s = 0;                                            // first lane of the current segment
            bool at_reset = false;                                    // the periodic reset at lane s is applied
            while (true) {
                if (!pending && !at_reset && RP > 0 && n0 + s > 0 && (n0 + s) % RP == 0) restart((uint32_t)(n0 + s));
                const float Qv0 = Qb - Qbc;
                const float Ql = Qv0 + sx, Al = Ab + sa;              // charge and |charge| after this lane's tick
                if (pending) {
                    const int32_t js = ns - n0;
                    if (js >= jn) break;                              // the sample is in a later chunk
                    const float Qv = lane_value(Ql, js), Av = lane_value(Al, js);
                    float qs = Qv;
                    if (P.sig_unc > 0.0f) qs += P.sig_unc * noise_normal(P, pid, (uint32_t)ns, ev, STREAM_SAMPLE);
                    const float xq = __fdiv_rn(qs, P.q_lsb);
                    const float fl = floorf(xq);
                    int32_t code = (int32_t)fmaxf(fminf(fl, 1.0e9f), -1.0e9f) + P.pedestal;
                    uint8_t flag = uncertain ? 2 : 0;
                    if (code < 0) { code = 0; flag |= 4; }
                    if (code > P.adc_max) { code = P.adc_max; flag |= 4; }
                    const float dist = (xq - fl) * P.q_lsb;
                    const float eps = P.eps_abs + P.eps_rel * (Av + fabsf(qs) + P.thr);
                    if (dist < eps || P.q_lsb - dist < eps) flag |= 1;
                    if (cnt < P.max_packets) {
                        if (lane == 0) {
                            pk_tick[obase + cnt] = ns;
                            pk_adc[obase + cnt] = (uint16_t)code;
                            pk_flag[obase + cnt] = flag;
                        }
                        ++cnt;
                    } else {
                        ++over;
                    }
                    restart((uint32_t)ns);
                    pending = false;
                    ready = ns + 1;
                    last = ns;
                    s = js + 1;
                    at_reset = false;
                    if (s >= jn) break;
                    scan(s);
                    continue;
                }
                // the next periodic reset after lane s ends the lanes compared against this segment's charge
                int32_t r = jn;
                if (RP > 0) {
                    const int32_t t = ((n0 + s) / RP + 1) * RP;       // first multiple of the period after n0 + s
                    if (t - n0 < jn) r = t - n0;
                }
                const int32_t lo = max(s, ready - n0);
                const bool cmp = lane >= lo && lane < r;
                float m = 0.0f, eps = 0.0f;
                if (cmp) {
                    float disc = 0.0f;
                    if (P.sig_disc > 0.0f && Ql + kNormalBound * P.sig_disc >= P.thr)
                        disc = P.sig_disc * noise_normal(P, pid, (uint32_t)n, ev, STREAM_DISC);
                    m = (Ql + disc) - P.thr;
                    eps = P.eps_abs + P.eps_rel * (Al + fabsf(Ql) + P.thr);
                }
                const uint64_t cross = __ballot(cmp && m >= 0.0f), near = __ballot(cmp && fabsf(m) < eps);
                if (cross) {
                    const int32_t c = __ffsll((unsigned long long)cross) - 1;
                    if (near & ((2ull << c) - 1)) uncertain = true;    // lanes up to the crossing (c = 63: all)
                    pending = true;
                    ns = max(n0 + c + P.hold, last + P.spacing);
                    if (ns >= NT) { ++dropped; done = true; break; }
                    continue;                                         // the sample may fall in this chunk
                }
                if (near) uncertain = true;
                if (r < jn) {                                         // periodic reset at lane r
                    restart((uint32_t)(n0 + r));
                    s = r;
                    at_reset = true;
                    scan(s);
                    continue;
                }
                break;
            }
            if (!done && s < jn) {                                    // carry the segment's charge into the next chunk
                const float y = lane_value(sx, jn - 1) - Qbc, t = Qb + y;
                Qbc = (t - Qb) - y;
                Qb = t;
                Ab += lane_value(sa, jn - 1);
            }
        }
        if (lane == 0) pk_cnt[slot] = off ? 0 : cnt;
        add_report(report, e, 2, rs, true);
        if (lane == 0 && dropped) {
            atomicAdd((unsigned long long *)&H->dropped, (unsigned long long)dropped);
            if (ev_cnt) atomicAdd((unsigned long long *)&ev_cnt[2 * e], (unsigned long long)dropped);
        }
        if (lane == 0 && over) {
            atomicAdd((unsigned long long *)&H->over, (unsigned long long)over);
            if (ev_cnt) atomicAdd((unsigned long long *)&ev_cnt[2 * e + 1], (unsigned long long)over);
        }
    }
}

void launch_electronics(const DevParams &P, const float *wave, const int32_t *slot_gp, const uint64_t *event_ids,
                        int64_t n_slots, const Work &w, hipStream_t st) {
    int64_t g = (n_slots + kWG / 64 - 1) / (kWG / 64);
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    k_electronics<<<(unsigned)g, kWG, 0, st>>>(P, wave, slot_gp, event_ids, w.n_ev, w.disabled, n_slots, w.pk_tick,
                                               w.pk_adc, w.pk_flag, w.pk_off, w.hdr, w.report, w.ev_cnt);
}

__global__ void k_compact(int32_t max_packets, int64_t n_slots, const int64_t *pk_off, const int32_t *slot_gp,
                          int32_t npx, const int32_t *pk_tick, const uint16_t *pk_adc, const uint8_t *pk_flag,
                          int32_t *o_pixel, int32_t *o_tick, uint16_t *o_adc, uint8_t *o_flag, int64_t cap) {
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= n_slots) return;
    const int64_t off = pk_off[slot], cnt = pk_off[slot + 1] - off;
    const int32_t pid = slot_gp[slot] % npx;
    for (int64_t k = 0; k < cnt && off + k < cap; ++k) {
        const int64_t src = slot * max_packets + k;
        o_pixel[off + k] = pid;
        o_tick[off + k] = pk_tick[src];
        o_adc[off + k] = pk_adc[src];
        o_flag[off + k] = pk_flag[src];
    }
}

__global__ void k_counts(int64_t n_slots, const int64_t *pk_off, const DevHeader *H, int64_t *counts, int64_t cap_pk,
                         int32_t n_ev, const int64_t *ev_pix_off, int64_t *ev_pkt_off) {
    const int64_t tot = pk_off[n_slots];
    if (threadIdx.x == 0 && blockIdx.x == 0 && counts) {
        counts[0] = n_slots;
        counts[1] = tot;
        counts[2] = H->dropped;
        counts[3] = H->over;
    }
    for (int e = threadIdx.x; ev_pkt_off && ev_pix_off && e <= n_ev; e += blockDim.x) ev_pkt_off[e] = pk_off[ev_pix_off[e]];
    (void)cap_pk;
}

void launch_compact_packets(const DevParams &P, const Work &w, int64_t n_slots, int32_t *pkt_pixel, int32_t *pkt_tick,
                            uint16_t *pkt_adc, uint8_t *pkt_flags, int64_t cap_packets, const int64_t *ev_pix_off,
                            int64_t *ev_pkt_off, int64_t *counts, hipStream_t st) {
    scan_exclusive<int64_t>(w.pk_off, n_slots + 1, w.scan_tmp, st);
    if (n_slots > 0)
        k_compact<<<(unsigned)((n_slots + kWG - 1) / kWG), kWG, 0, st>>>(P.max_packets, n_slots, w.pk_off, w.slot_gp,
                                                                         P.npx, w.pk_tick, w.pk_adc, w.pk_flag, pkt_pixel,
                                                                         pkt_tick, pkt_adc, pkt_flags, cap_packets);
    k_counts<<<1, kWG, 0, st>>>(n_slots, w.pk_off, w.hdr, counts, cap_packets, w.n_ev, ev_pix_off, ev_pkt_off);
}

// ================================================================================================= work statistics
// Algorithmic work of the induction stage of the last pipeline call: for every (segment, pixel) pair, the number of
// charge cells in the pixel's table reach and the number of (cell, tick) products that land in the tick window.
__global__ void k_work_stats(DevParams P, const SegInfo *si, int64_t n_seg, unsigned long long *acc) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_seg) return;
    const SegInfo g = si[s];
    if (g.n_pairs == 0) return;
    // kept table ticks summed over the segment's cell ticks a (independent of the pixel)
    unsigned long long kept = 0;
    for (int32_t a = g.a0; a < g.a0 + g.na; ++a) {
        const int32_t lo = max(a - P.t_r + 1, 0), hi = min(a, P.nticks - 1);
        if (hi >= lo) kept += (unsigned long long)(hi - lo + 1);
    }
    unsigned long long cols = 0;
    for (int32_t iy = g.iy0; iy <= g.iy1; ++iy)
        for (int32_t ix = g.ix0; ix <= g.ix1; ++ix) {
            const int32_t uc = ix * P.nsub + P.nsub / 2, vc = iy * P.nsub + P.nsub / 2;
            const int32_t nu = min(g.u0 + g.nu - 1, uc + P.bx - 1) - max(g.u0, uc - P.bx) + 1;
            const int32_t nv = min(g.v0 + g.nv - 1, vc + P.by - 1) - max(g.v0, vc - P.by) + 1;
            if (nu > 0 && nv > 0) cols += (unsigned long long)nu * nv;
        }
    atomicAdd(&acc[0], (unsigned long long)g.n_pairs);
    atomicAdd(&acc[1], cols * kept);
    atomicAdd(&acc[2], cols * (unsigned long long)g.na);
    atomicAdd(&acc[3], (unsigned long long)g.nu * g.nv * g.na);
}

void launch_work_stats(const DevParams &P, const SegInfo *si, int64_t n_seg, unsigned long long *acc, hipStream_t st) {
    if (n_seg > 0) k_work_stats<<<(unsigned)((n_seg + kWG - 1) / kWG), kWG, 0, st>>>(P, si, n_seg, acc);
}

// Summed induction: per active pixel, the (column-piece tick, table tick) products that land in the window.
// Summed mode: a tick of a piece counts only if it holds charge (the ticks a piece adds for alignment, and the short
// gaps between segments that a piece spans, hold exact zeros and are not algorithmic work).
__global__ void k_work_stats_summed(DevParams P, int64_t n_slots, const int64_t *list_off, const PieceRef *rec,
                                    const float *S, const int64_t *mlist_off, const PieceRef *mrec, int32_t tile,
                                    unsigned long long *acc) {
    int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= n_slots) return;
    unsigned long long f = 0, cells = 0, issued = 0;
    const int32_t n_tiles = (P.nticks + tile - 1) / tile;
    // algorithmic work: every non-zero summed charge tick of every column piece in reach, times the table ticks
    // that land inside the readout
    for (int64_t q = list_off[slot]; q < list_off[slot + 1]; ++q) {
        const PieceRef g = rec[q];
        const float *sv = S + (int64_t)g.cell8 * kAC;
        for (int32_t a = g.a0; a < g.a0 + g.na; ++a) {
            if (sv[a - g.a0] == 0.0f) continue;
            const int32_t lo = max(a - P.t_r + 1, 0), hi = min(a, P.nticks - 1);
            if (hi >= lo) f += (unsigned long long)(hi - lo + 1);
            ++cells;
        }
    }
    // products the summed kernel computes for the merged records, zeros included: every tile (of `tile` ticks) a
    // record's window meets, all its ticks x every 8-tick charge block
    for (int64_t q = mlist_off[slot]; q < mlist_off[slot + 1]; ++q) {
        const PieceRef g = mrec[q];
        const int32_t t_lo = max(floor_div(g.a0 - P.t_r + 1, tile), 0);
        const int32_t t_hi = min(floor_div(g.a0 + g.na - 1, tile), n_tiles - 1);
        if (t_hi >= t_lo)
            issued += (unsigned long long)(t_hi - t_lo + 1) * (unsigned long long)((g.na + kAC - 1) / kAC) *
                      (unsigned long long)(tile * kAC);
    }
    atomicAdd(&acc[0], (unsigned long long)(mlist_off[slot + 1] - mlist_off[slot]));
    atomicAdd(&acc[1], f);
    atomicAdd(&acc[2], cells);
    atomicAdd(&acc[3], issued);
}

void launch_work_stats_summed(const DevParams &P, int64_t n_slots, const int64_t *list_off, const PieceRef *rec,
                              const float *S, const int64_t *mlist_off, const PieceRef *mrec, bool tile256,
                              unsigned long long *acc, hipStream_t st) {
    if (n_slots > 0)
        k_work_stats_summed<<<(unsigned)((n_slots + kWG - 1) / kWG), kWG, 0, st>>>(
            P, n_slots, list_off, rec, S, mlist_off, mrec, tile256 ? kTile4 : kTileTicks, acc);
}

// ================================================================================================= Philox test hook
__global__ void k_philox(const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint4 c = make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
    uint4 x = philox4x32_10(c, k0, k1);
    out[4 * i] = x.x; out[4 * i + 1] = x.y; out[4 * i + 2] = x.z; out[4 * i + 3] = x.w;
}

void launch_philox(const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out, int64_t n, hipStream_t st) {
    if (n > 0) k_philox<<<(unsigned)((n + kWG - 1) / kWG), kWG, 0, st>>>(ctr, k0, k1, out, n);
}

}  // namespace ltsim
