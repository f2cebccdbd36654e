// device.hpp -- types and device helpers shared by the gfx950 kernels of libltsim.
//
// Precision scheme: all bulk arithmetic is FP32.  The library is compiled with -ffp-contract=off; multiply-adds
// that should be fused are written as fmaf.  Coordinates are never used in absolute FP32 form where a
// rounding of the absolute value would move charge relative to the sub-pixel or tick grid: each segment gets an
// integer reference bin / tick and an FP32 offset from it, computed once per segment with error-free
// transformations (two-sum / two-product on FP32 hi/lo pairs), so that offsets are accurate to ~1e-9 cm and
// ~1e-8 us whatever the tile coordinate.  FP64 is used only for the per-event charge report.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ltsim {

constexpr int kWG = 256;             // threads per workgroup of the per-pixel / per-segment kernels
constexpr int kNaMax = 256;          // maximum charge-box extent in ticks per segment
constexpr int kBoxMax = 256;         // maximum charge-box extent in sub-pixel bins per axis
constexpr int kAC = 8;               // cell ticks per register block in the induction inner loop
constexpr int kRTMax = 8;            // ticks per thread in the induction inner loop (max)
constexpr int kTileTicks = 512;      // ticks of one wavefront work unit of the summed induction (64 lanes x 8)
constexpr int kPieceMax = 248;       // maximum ticks of a summed charge column piece
// Zero padding on each side of every table column.  The per-pair induction reads at most kNaMax + 16 values below
// and kNaMax + 8 above the table span; the summed induction's tiles overhang a column's tick window by up to
// kTileTicks - 1 ticks, so it reads at most kTileTicks + kPieceMax + 16 below and kTileTicks + kPieceMax above.
constexpr int kPad = 792;
static_assert(kPad % 8 == 0, "table columns keep 32-byte alignment");
static_assert(kPad >= kNaMax + 16, "per-pair induction reads");
static_assert(kPad >= kTileTicks + kPieceMax + 16, "summed induction reads");
constexpr int kMaxTicks = 16384;
constexpr int kCellSlack = 2 * kAC;  // floats allocated past the last cell: the induction loop loads one block ahead
constexpr float kNormalBound = 6.7638f;  // |Box-Muller normal| <= sqrt(-2 ln 2^-33) = 6.76372 for u >= 2^-33

enum : int32_t { SEG_BOX_CLAMP = 1, SEG_INVALID = 2, SEG_TOO_LONG = 4, SEG_STRADDLE = 8 };
enum : int32_t { ST_INVALID = 1, ST_TOO_LONG = 2, ST_CAPACITY = 4 };
enum : uint32_t { STREAM_DISC = 0, STREAM_RESET = 1, STREAM_SAMPLE = 2, STREAM_MC = 3 };
constexpr uint32_t kTickInitial = 0xFFFFFFFFu;

// Derived constants, FP32 (hi/lo pairs where an absolute coordinate is involved).
struct DevParams {
    // recombination / drift (Sec. 3.1, 3.2)
    int32_t recomb_model;
    float birks_ab, birks_kb_eps, box_alpha, box_beta_eps, inv_w_ion;
    float inv_vd_hi, inv_vd_lo, inv_lifetime, two_dl, two_dt, za_hi, za_lo;
    float step, nsig, inv_norm;             // inv_norm = 1 / P(|g| <= n_sigma)
    int32_t cell_pad;                       // charge-cell rows rounded up to a multiple of this many ticks (kAC for
                                            // the per-pair kernels' 8-tick blocks, 1 for the summed columns)
    int32_t mc_draws;                       // 0: expectation over the diffusion draws; M > 0: M draws per point
    int32_t per_point;                      // lifetime and diffusion at each sample point (1) or the midpoint (0)
    // grid
    float b_hi, b_lo, x0_hi, x0_lo, y0_hi, y0_lo, tick_hi, tick_lo, tb_hi, tb_lo;
    int32_t nx, ny, nsub, nticks, npx;
    // field-response table
    int32_t t_r, bx, by, col_len;           // col_len = kPad + t_r rounded up to 8 + kPad
    // electronics (Sec. 3.4)
    float thr, q_lsb, sig_reset, sig_disc, sig_unc;
    int32_t hold, spacing, pedestal, adc_max, max_packets, reset_period;
    uint32_t key0, key1;
    float eps_rel, eps_abs;
};

// One segment after recombination, drift and rasterisation (Sec. 3.1-3.3).
struct alignas(16) SegInfo {
    float q_r, q_a, q_pt, t_drift;          // electrons after recombination / lifetime; per sample point; us
    float sigma_t, sigma_time, dedx, _f0;   // cm, us, MeV/cm
    float ox, oy, ot, _f1;                  // start-point offsets from its reference bin / tick lower edge
    float dx, dy, dta, zz0;                 // segment deltas (x, y, linear arrival time), z0 - z_anode
    float dz, dt, _f3, _f4;
    int32_t u_ref, v_ref, a_ref, n_points;  // reference bin / tick of the start point
    int32_t u0, nu, v0, nv;                 // charge box, absolute sub-pixel bin indices
    int32_t a0, na, na_pad, flags;          // charge box, absolute tick indices (na_pad = na rounded up to cell_pad)
    int32_t ix0, ix1, iy0, iy1;             // pixel rectangle reached (clipped to the grid; empty if ix1 < ix0)
    int32_t event, n_pairs, _i0, _i1;
    int64_t cell_off, _l0;
};
static_assert(sizeof(SegInfo) == 176, "SegInfo layout");

// Device-resident totals of one pipeline invocation.
struct DevHeader {
    int64_t n_pairs, n_slots, n_cells, n_packets;
    int64_t dropped, over;
    int64_t n_colseg;                       // sum over segments of nu * nv (bound for the summed induction)
    uint32_t work[4];                       // dynamic work counters of persistent kernels
    int32_t status;                         // ST_* bits
    int32_t _pad[3];
};

// ------------------------------------------------------------------------------------------------ helpers
__device__ __forceinline__ int32_t fold(int32_t k) { return k >= 0 ? k : -k - 1; }

__device__ __forceinline__ int32_t floor_div(int32_t a, int32_t b) {  // b > 0
    return a >= 0 ? a / b : -((-a + b - 1) / b);
}
__device__ __forceinline__ int32_t ceil_div(int32_t a, int32_t b) {   // b > 0
    return a >= 0 ? (a + b - 1) / b : -((-a) / b);
}

// error-free transformations (Knuth two-sum)
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
    s = __fadd_rn(a, b);
    float bb = __fsub_rn(s, a);
    e = __fadd_rn(__fsub_rn(a, __fsub_rn(s, bb)), __fsub_rn(b, bb));
}

// Split the double-float value (vh + vl) - (oh + ol) into k * step + off with off in [0, step), step = sh + sl.
__device__ __forceinline__ void ref_offset(float vh, float vl, float oh, float ol, float sh, float sl,
                                           int32_t &k, float &off) {
    float dh, e1;
    two_sum(vh, -oh, dh, e1);
    float dl = __fadd_rn(__fsub_rn(e1, ol), vl);
    float kf = floorf(__fdiv_rn(dh, sh));
    float p = __fmul_rn(kf, sh);
    float pe = fmaf(kf, sh, -p);                      // kf*sh = p + pe exactly
    off = __fadd_rn(__fsub_rn(__fsub_rn(dh, p), pe), __fsub_rn(dl, __fmul_rn(kf, sl)));
    k = (int32_t)kf;
    if (off < 0.0f) { k -= 1; off = __fadd_rn(off, sh); }
    else if (off >= sh) { k += 1; off = __fsub_rn(off, sh); }
}

// Local position of sample point mu (of N) relative to the segment's reference bin / tick edges.  The same
// function (same operation sequence) serves the charge-box bounds and the charge cells.
__device__ __forceinline__ void point_local(const SegInfo &g, const DevParams &P, int32_t mu, float &lx, float &ly,
                                            float &lt) {
    float s = __fdiv_rn((float)mu + 0.5f, (float)g.n_points);
    lx = fmaf(s, g.dx, g.ox);
    ly = fmaf(s, g.dy, g.oy);
    if (g.flags & SEG_STRADDLE) {
        float d = __fsub_rn(fabsf(fmaf(s, g.dz, g.zz0)), fabsf(g.zz0));
        lt = fmaf(d, P.inv_vd_hi, fmaf(s, g.dt, g.ot));
    } else {
        lt = fmaf(s, g.dta, g.ot);
    }
}

// ------------------------------------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, two 32x32->64 products per round, key bumped by
// the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Standard normal for (pixel, tick, event, stream): Box-Muller on the first two words.  Counter layout:
// (pixel id, tick, event id low word, (event id high word << 4) | stream).
__device__ __forceinline__ float noise_normal(const DevParams &P, uint32_t pixel, uint32_t tick, uint64_t event,
                                              uint32_t stream) {
    uint4 c = make_uint4(pixel, tick, (uint32_t)event, (uint32_t)((event >> 32) << 4) | (stream & 15u));
    uint4 x = philox4x32_10(c, P.key0, P.key1);
    float u0 = fmaf((float)x.x, 0x1p-32f, 0x1p-33f);
    float u1 = fmaf((float)x.y, 0x1p-32f, 0x1p-33f);
    return sqrtf(-2.0f * logf(u0)) * cospif(2.0f * u1);
}

// Drift of sample point mu at its own drift time (per-point mode): charge Q_R / N * exp(-t / tau) and the
// transverse / arrival-time widths sqrt(2 D t).
__device__ __forceinline__ void point_drift(const SegInfo &g, const DevParams &P, int32_t mu, float &q, float &sT,
                                            float &sL) {
    const float s = __fdiv_rn((float)mu + 0.5f, (float)g.n_points);
    const float td = fabsf(fmaf(s, g.dz, g.zz0)) * P.inv_vd_hi;
    q = (g.q_r / (float)g.n_points) * expf(-td * P.inv_lifetime);
    sT = sqrtf(P.two_dt * td);
    sL = sqrtf(P.two_dl * td) * P.inv_vd_hi;
}

// Diffusion perturbation of draw `draw` (= point * M + m) of segment `seg` of an event (Monte Carlo form of
// eq. (rho)): the cosine and sine Box-Muller branches of words (0, 1) give the x and y normals, the cosine branch of
// words (2, 3) the arrival-time normal.  Each normal is truncated to |g| <= n_sigma: a component outside is replaced
// by the same component of the next try (try r uses stream 3 + r, nine tries; none accepted leaves 0).
constexpr int kMcTries = 9;
__device__ __forceinline__ void mc_normals(const DevParams &P, uint32_t seg, uint32_t draw, uint64_t event, float &gx,
                                           float &gy, float &gt) {
    gx = gy = gt = 0.0f;
    bool hx = false, hy = false, ht = false;
    for (uint32_t r = 0; r < (uint32_t)kMcTries && !(hx && hy && ht); ++r) {
        const uint4 c = make_uint4(seg, draw, (uint32_t)event, (uint32_t)((event >> 32) << 4) | ((STREAM_MC + r) & 15u));
        const uint4 x = philox4x32_10(c, P.key0, P.key1);
        const float r0 = sqrtf(-2.0f * logf(fmaf((float)x.x, 0x1p-32f, 0x1p-33f)));
        const float a0 = 2.0f * fmaf((float)x.y, 0x1p-32f, 0x1p-33f);
        const float r1 = sqrtf(-2.0f * logf(fmaf((float)x.z, 0x1p-32f, 0x1p-33f)));
        const float a1 = 2.0f * fmaf((float)x.w, 0x1p-32f, 0x1p-33f);
        const float cx = r0 * cospif(a0), cy = r0 * sinpif(a0), ct = r1 * cospif(a1);
        if (!hx && fabsf(cx) <= P.nsig) { gx = cx; hx = true; }
        if (!hy && fabsf(cy) <= P.nsig) { gy = cy; hy = true; }
        if (!ht && fabsf(ct) <= P.nsig) { gt = ct; ht = true; }
    }
}

// Index of the bin of local coordinate y on a grid of edges k * (wh + wl) (the same edge expression as the bin
// masses use), from a first guess by division.
__device__ __forceinline__ int32_t local_bin(float y, float wh, float wl) {
    float kf = floorf(__fdiv_rn(y, wh));
    if (__fadd_rn(fmaf(kf, wh, -y), __fmul_rn(kf, wl)) > 0.0f) {
        kf -= 1.0f;
    } else {
        const float k1 = kf + 1.0f;
        if (__fadd_rn(fmaf(k1, wh, -y), __fmul_rn(k1, wl)) <= 0.0f) kf = k1;
    }
    return (int32_t)kf;
}

// ------------------------------------------------------------------------------------------------ Gaussian
// Tail beyond |z| of the standard normal, z clamped to the truncation n: erfc(|z| / sqrt 2) / 2.
__device__ __forceinline__ float tail(float z) { return 0.5f * erfcf(fabsf(z) * 0.70710678118654752f); }

// Truncated, renormalised mass between standardised edges za <= zb (both clamped to [-n, n]) given their tails,
// evaluated on the side away from the mean to avoid cancellation.
__device__ __forceinline__ float tmass(float za, float ta, float zb, float tb, float inv_norm) {
    float m;
    if (za >= 0.0f) m = ta - tb;
    else if (zb <= 0.0f) m = tb - ta;
    else m = (1.0f - tb) - ta;
    return fmaxf(m, 0.0f) * inv_norm;
}

}  // namespace ltsim
