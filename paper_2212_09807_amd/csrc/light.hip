// light.hip -- light path of the simulation (Sec. 4.2, 4.3) on given photocurrents, for gfx950, with its C ABI.
//
//   mu[d][t] = sum_{k=0}^{K-1} ipe[d][t-k] * w[k],  w[k] = tick * f_scint(k * tick)      (FP64, truncated direct)
//   pe[d][t] = Poisson(mu) by inverse transform sampling, or mu + sqrt(mu) g above normal_above   (FP64)
//   V[d][t]  = G * sum_{k<R} pe[d][t-k] * r[k] + sum_{f=1}^{F} A_f cos(2 pi f t / T + phi_{d,f})   (FP32)
//   triggers per detector group on the summed V (threshold, dead time)
//
// The scintillation sum runs in FP64 because the photoelectron counts are integers decided by comparing a uniform
// variate with cumulative Poisson probabilities of mu: an FP32 mean (a sum of ~8000 products) would move those
// boundaries by ~1e-6 and flip counts, while FP64 leaves them where an FP64 evaluation puts them (the FP64 vector
// rate of gfx950 equals its non-packed FP32 rate).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "device.hpp"
#include "../../include/ltsim.h"
#include "api.hpp"

namespace ltsim {
namespace {

constexpr int kLWG = 256;            // threads per workgroup
constexpr int kLRT = 8;              // ticks per thread in the convolutions
constexpr int kLTile = kLWG * kLRT;  // ticks per workgroup tile
constexpr uint32_t kStreamLightPe = 12u, kStreamLightNoise = 13u;

typedef const double __attribute__((address_space(4))) *cdouble_ptr;
typedef const float __attribute__((address_space(4))) *cfloat4_ptr;

// mu for 8 consecutive ticks per lane; xp holds one row per detector with stride Ks (a multiple of 8 floats): Kp =
// 8 nkb + 8 zeros in front, the photocurrent at Kp + t, zeros up to the stride.  w is the kernel padded with zeros
// to nkb * 8 taps.  A workgroup covers 512 ticks of one detector; its four wavefronts take a quarter of the tap
// blocks each, and their partial sums are added in wavefront order through LDS (fixed order: deterministic).  Tap
// block kb needs x[t0 - 8kb - 7 .. t0 - 8kb + 7]: its 8-value half b_kb = x[t0 - 8kb .. +7] and the upper seven
// values of b_{kb+1}, so the blocks go in ping-pong through two 8-value register sets, each half loaded (two aligned
// 16-byte loads) and converted to FP64 once.  Reads past a row's end see its zero tail or the next row's zeros and
// only reach ticks >= T, which are not stored.
constexpr int kLScintTicks = 64 * kLRT;   // ticks per workgroup of the scintillation sum

__global__ __launch_bounds__(kLWG) void k_light_scint(const float *__restrict__ xp, int32_t Kp, int32_t Ks, int32_t T,
                                                      const double *__restrict__ w, int32_t nkb, double *__restrict__ mu) {
    __shared__ double part[kLWG / 64 - 1][64][kLRT + 1];
    const int32_t d = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int32_t wv = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
    const int32_t t0 = blockIdx.x * kLScintTicks + lane * kLRT;
    const float *x = xp + (int64_t)d * Ks + Kp + t0;
    cdouble_ptr wc = (cdouble_ptr)w;
    auto load = [](const float *p, double (&v)[8]) {
        const float4 lo = *(const float4 *)p, hi = *(const float4 *)(p + 4);
        v[0] = lo.x; v[1] = lo.y; v[2] = lo.z; v[3] = lo.w; v[4] = hi.x; v[5] = hi.y; v[6] = hi.z; v[7] = hi.w;
    };
    double acc[kLRT];
#pragma unroll
    for (int r = 0; r < kLRT; ++r) acc[r] = 0.0;
    // acc[r] += w[8kb + q] * x[t0 + r - q - 8kb]: from b_kb when r >= q, else from b_{kb+1}
    auto block = [&](int32_t kb, const double (&B)[8], const double (&N)[8]) {
        double wk[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) wk[q] = wc[8 * kb + q];
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int r = 0; r < kLRT; ++r) acc[r] = fma(wk[q], r >= q ? B[r - q] : N[8 + r - q], acc[r]);
    };
    const int32_t nq = (nkb + 3) / 4, kb0 = wv * nq, kb1 = min(kb0 + nq, nkb);
    if (t0 < T && kb0 < kb1) {
        double X[8], Y[8];
        load(x - 8 * kb0, X);
        for (int32_t kb = kb0; kb < kb1; kb += 2) {
            load(x - 8 * (kb + 1), Y);
            block(kb, X, Y);
            if (kb + 1 >= kb1) break;
            load(x - 8 * (kb + 2), X);
            block(kb + 1, Y, X);
        }
    }
    if (wv > 0)
#pragma unroll
        for (int r = 0; r < kLRT; ++r) part[wv - 1][lane][r] = acc[r];
    __syncthreads();
    if (wv == 0 && t0 < T) {
#pragma unroll
        for (int k = 0; k < kLWG / 64 - 1; ++k)
#pragma unroll
            for (int r = 0; r < kLRT; ++r) acc[r] += part[k][lane][r];
        double *o = mu + (int64_t)d * T + t0;
#pragma unroll
        for (int r = 0; r < kLRT; ++r)
            if (t0 + r < T) o[r] = acc[r];
    }
}

__global__ void k_light_pad(const float *__restrict__ ipe, float *__restrict__ xp, int32_t Kp, int32_t Ks, int32_t T,
                            int32_t n_det) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_det * T) return;
    const int64_t d = i / T, t = i - d * T;
    xp[d * Ks + Kp + t] = ipe[i];
}

// Photoelectron statistics; writes pe (FP64) and the FP32 copy with Rp zeros in front for the response sum.
__global__ void k_light_fluct(const double *__restrict__ mu, double *__restrict__ pe, float *__restrict__ pef,
                              int32_t Rp, int32_t T, int32_t n_det, uint64_t event, uint32_t k0, uint32_t k1,
                              double normal_above) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_det * T) return;
    const int64_t d = i / T, t = i - d * T;
    const uint4 c = make_uint4((uint32_t)d, (uint32_t)t, (uint32_t)event, (uint32_t)((event >> 32) << 4) | kStreamLightPe);
    const uint4 x = philox4x32_10(c, k0, k1);
    const double u = ((double)x.x + 0.5) * 0x1p-32;
    const double m = mu[i];
    double n;
    if (m > normal_above) {
        const double u1 = ((double)x.y + 0.5) * 0x1p-32;
        n = m + sqrt(m) * (sqrt(-2.0 * log(u)) * cos(6.283185307179586477 * u1));
    } else {
        double p = exp(-m), F = p;
        int32_t k = 0;
        while (u > F && k < 1000) {
            ++k;
            p *= m / k;
            F += p;
        }
        n = (double)k;
    }
    pe[i] = n;
    pef[d * (Rp + T) + Rp + t] = (float)n;
}

// Noise coefficients per (detector, frequency): A_f cos(phi), A_f sin(phi), phi = 2 pi u.
__global__ void k_light_noise_coef(const float *__restrict__ amp, int32_t F, int32_t n_det, uint64_t event, uint32_t k0,
                                   uint32_t k1, float2 *__restrict__ coef) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_det * F) return;
    const int32_t d = (int32_t)(i / F), f = (int32_t)(i - (int64_t)d * F) + 1;
    const uint4 c = make_uint4((uint32_t)d, (uint32_t)f, (uint32_t)event, (uint32_t)((event >> 32) << 4) | kStreamLightNoise);
    const uint4 x = philox4x32_10(c, k0, k1);
    const double phi = 6.283185307179586477 * (((double)x.x + 0.5) * 0x1p-32);
    coef[i] = make_float2((float)(amp[f - 1] * cos(phi)), (float)(amp[f - 1] * sin(phi)));
}

// Noise by FFT (power-of-two windows, T >= 4, whose complex spectrum and a quarter-period cosine table fit in LDS):
// noise[t] is the real part of y[t] = sum_{f=1}^{F} A_f e^{i phi_f} e^{2 pi i f t / T}, an unnormalised inverse DFT of
// the one-sided spectrum, computed in place by iterative radix-2 decimation in time (bit-reversed load, log2 T
// butterfly stages).  The twiddles e^{2 pi i m / T}, m < T/2, come from cos(2 pi m / T) for m <= T/4 staged in LDS:
// sin(2 pi m / T) = cos(2 pi (T/4 - m) / T), and past a quarter period cos and sin follow from the quarter shift.
// One workgroup per detector.
inline size_t noise_fft_lds(size_t T) { return sizeof(float2) * T + sizeof(float) * (T / 4 + 1); }

__global__ __launch_bounds__(1024) void k_light_noise_fft(const float2 *__restrict__ coef, int32_t F, int32_t T,
                                                          int32_t log2T, const float *__restrict__ Ct,
                                                          float *__restrict__ nz) {
    extern __shared__ float2 xs[];
    float *qc = (float *)(xs + T);
    const int32_t d = blockIdx.x;
    const int32_t Q = T >> 2;
    const float2 *cf = coef + (int64_t)d * F;
    for (int32_t i = threadIdx.x; i < T; i += blockDim.x) {
        const float2 y = (i >= 1 && i <= F) ? cf[i - 1] : make_float2(0.0f, 0.0f);
        xs[__builtin_bitreverse32((uint32_t)i) >> (32 - log2T)] = y;
    }
    for (int32_t m = threadIdx.x; m <= Q; m += blockDim.x) qc[m] = Ct[m];
    __syncthreads();
    for (int32_t half = 1; half < T; half <<= 1) {
        const int32_t stride = T / (2 * half);                    // twiddle index step for this stage
        for (int32_t k = threadIdx.x; k < T / 2; k += blockDim.x) {
            const int32_t j = k & (half - 1);
            const int32_t i0 = ((k - j) << 1) + j, i1 = i0 + half;
            const int32_t m = j * stride;                         // < T / 2
            float wr, wi;
            if (m <= Q) {
                wr = qc[m];
                wi = qc[Q - m];
            } else {
                wr = -qc[T / 2 - m];
                wi = qc[m - Q];
            }
            const float2 a = xs[i0], b = xs[i1];
            const float tr = wr * b.x - wi * b.y, ti = fmaf(wr, b.y, wi * b.x);
            xs[i0] = make_float2(a.x + tr, a.y + ti);
            xs[i1] = make_float2(a.x - tr, a.y - ti);
        }
        __syncthreads();
    }
    float *o = nz + (int64_t)d * T;
    for (int32_t i = threadIdx.x; i < T; i += blockDim.x) o[i] = xs[i].x;
}

// V for 8 consecutive ticks per thread: the response sum (pef row with Rp zeros in front, r padded to nrb * 8 taps)
// and the noise sinusoids: cos(2 pi f t / T + phi) = C[m] cos(phi) - S[m] sin(phi), m = f t mod T, with the angle of
// the following ticks advanced by the rotation (C[f], S[f]).
__global__ __launch_bounds__(kLWG) void k_light_response(const float *__restrict__ pef, int32_t Rp, int32_t T,
                                                         const float *__restrict__ r, int32_t nrb, float gain,
                                                         const float2 *__restrict__ coef, int32_t F,
                                                         const float *__restrict__ Ct, const float *__restrict__ St,
                                                         const float *__restrict__ nzpre, float *__restrict__ V) {
    const int32_t d = blockIdx.y;
    const int32_t t0 = blockIdx.x * kLTile + threadIdx.x * kLRT;
    if (t0 >= T) return;
    const float *x = pef + (int64_t)d * (Rp + T) + Rp + t0 - 7;
    cfloat4_ptr rc = (cfloat4_ptr)r;
    float acc[kLRT];
#pragma unroll
    for (int j = 0; j < kLRT; ++j) acc[j] = 0.0f;
    for (int32_t kb = 0; kb < nrb; ++kb) {
        float win[kLRT + 7];
#pragma unroll
        for (int m = 0; m < kLRT + 7; ++m) win[m] = x[m - 8 * kb];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float rk = rc[8 * kb + q];
#pragma unroll
            for (int j = 0; j < kLRT; ++j) acc[j] = fmaf(rk, win[j - q + 7], acc[j]);
        }
    }
    float nz[kLRT];
#pragma unroll
    for (int j = 0; j < kLRT; ++j) nz[j] = (nzpre && t0 + j < T) ? nzpre[(int64_t)d * T + t0 + j] : 0.0f;
    const float2 *cf = coef + (int64_t)d * F;
    int32_t m0 = 0;                                    // f * t0 mod T, advanced by t0 per frequency
    for (int32_t f = 1; f <= (nzpre ? 0 : F); ++f) {
        const float2 ab = cf[f - 1];
        m0 += t0;
        if (m0 >= T) m0 -= T;
        float c = Ct[m0], s = St[m0];
        const float c1 = Ct[f], s1 = St[f];
#pragma unroll
        for (int j = 0; j < kLRT; ++j) {
            nz[j] = fmaf(ab.x, c, fmaf(-ab.y, s, nz[j]));
            const float cn = fmaf(c, c1, -s * s1);
            s = fmaf(s, c1, c * s1);
            c = cn;
        }
    }
    float *o = V + (int64_t)d * T + t0;
#pragma unroll
    for (int j = 0; j < kLRT; ++j)
        if (t0 + j < T) o[j] = fmaf(gain, acc[j], nz[j]);
}

// Triggers per detector group, in two kernels.  k_light_trigger_masks: one thread per (group, tick) sums the
// group's waveforms (fixed detector order), and each wavefront's ballot is the mask of that 64-tick chunk's ticks
// that reach the threshold.  k_light_trigger_scan: one workgroup per group stages the group's chunk masks in LDS,
// then one thread walks the non-empty ones in time order: the first set bit at or after the end of the dead time
// triggers, and the dead time restarts from it.
__global__ __launch_bounds__(256) void k_light_trigger_masks(const float *__restrict__ V, int32_t T, int32_t group,
                                                             float thr, uint64_t *__restrict__ masks) {
    const int32_t g = blockIdx.y;
    const int32_t nch = (T + 63) / 64;
    const int32_t t = blockIdx.x * 256 + threadIdx.x;
    float s = 0.0f;
    if (t < T)
        for (int32_t k = 0; k < group; ++k) s += V[(int64_t)(g * group + k) * T + t];
    const uint64_t m = __ballot(t < T && s >= thr);
    if ((threadIdx.x & 63) == 0 && t / 64 < nch) masks[(int64_t)g * nch + t / 64] = m;
}

__global__ __launch_bounds__(256) void k_light_trigger_scan(const uint64_t *__restrict__ masks, int32_t T,
                                                            int32_t dead, int32_t max_trig, int32_t *__restrict__ trig,
                                                            int32_t *__restrict__ count) {
    extern __shared__ uint64_t mk[];
    const int32_t g = blockIdx.x;
    const int32_t nch = (T + 63) / 64;
    for (int32_t c = threadIdx.x; c < nch; c += blockDim.x) mk[c] = masks[(int64_t)g * nch + c];
    __syncthreads();
    if (threadIdx.x >= 64) return;
    // the first wavefront finds the chunks with any tick over threshold, 64 chunks per ballot; lane 0 walks only
    // those, in time order
    const int lane = threadIdx.x;
    int32_t ready = 0, n = 0;
    for (int32_t c0 = 0; c0 < nch && n < max_trig; c0 += 64) {
        uint64_t any = __ballot(c0 + lane < nch && mk[c0 + lane] != 0);
        if (lane == 0) {
            while (any && n < max_trig) {
                const int32_t c = c0 + __builtin_ctzll(any);
                any &= any - 1;
                uint64_t m = mk[c];
                for (;;) {
                    const int32_t off = ready - 64 * c;          // ticks of this chunk still in the dead time
                    if (off >= 64) break;
                    if (off > 0) m &= ~((1ull << off) - 1ull);
                    if (m == 0 || n >= max_trig) break;
                    const int32_t tf = 64 * c + __builtin_ctzll(m);
                    trig[(int64_t)g * max_trig + n++] = tf;
                    ready = tf + dead;
                }
            }
        }
        n = __shfl(n, 0);
        ready = __shfl(ready, 0);
    }
    if (lane != 0) return;
    for (int32_t i = n; i < max_trig; ++i) trig[(int64_t)g * max_trig + i] = -1;
    count[g] = n;
}

template <typename T>
struct DBuf {
    T *p = nullptr;
    ~DBuf() { if (p) (void)hipFree(p); }
    hipError_t alloc(size_t n) { return hipMalloc((void **)&p, sizeof(T) * std::max<size_t>(n, 1)); }
};

}  // namespace
}  // namespace ltsim

using namespace ltsim;

struct lts_light {
    lts_light_params p{};
    int device = 0;
    int32_t K = 0, nkb = 0, Kp = 0, Ks = 0, R = 0, nrb = 0, Rp = 0, F = 0;
    uint32_t k0 = 0, k1 = 0;
    bool sticky = false;
    std::string err;
    DBuf<double> w, mu, pe;
    DBuf<float> xp, pef, r, amp, Ct, St;
    DBuf<float2> coef;
    DBuf<uint64_t> tmask;                            // trigger chunk masks [group][64-tick chunk]
    DBuf<float> nz;                                  // noise by FFT (when fft_log2 > 0)
    int32_t fft_log2 = 0;
    // replay through a HIP graph: captured once per set of caller buffers, the event id set per call in the two
    // kernel nodes that draw random numbers
    bool use_graph = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    // two instances used in turn: an instance is re-parameterised only after its previous launch has finished
    // (its event), so one call's graph can still run while the next call sets up the other
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipEvent_t done[2] = {nullptr, nullptr};
    bool launched[2] = {false, false};
    int32_t turn = 0;
    hipGraphNode_t fluct_node = nullptr, coef_node = nullptr;
    const void *g_ptrs[6] = {};
};

namespace {
lts_status lfail(lts_light *L, lts_status s, const std::string &m) {
    if (L) {
        L->err = m;
        if (s == LTS_ERR_DEVICE) L->sticky = true;
    }
    return s;
}
#define LHIP(L, call)                                                                                         \
    do {                                                                                                      \
        hipError_t e_ = (call);                                                                               \
        if (e_ != hipSuccess) return lfail(L, e_ == hipErrorOutOfMemory ? LTS_ERR_OOM : LTS_ERR_DEVICE,       \
                                          std::string(#call) + ": " + hipGetErrorString(e_));                 \
    } while (0)
}  // namespace

namespace {

// The kernel sequence of one light event on stream st (shapes fixed by the simulator's parameters).
void launch_light(lts_light *L, uint64_t event_id, const float *ipe, double *mu_d, double *pe_d, float *V,
                  int32_t *trig, int32_t *trig_count, hipStream_t st) {
    const lts_light_params &q = L->p;
    const int32_t T = q.n_ticks, nd = q.n_det;
    const int64_t n = (int64_t)nd * T;
    const unsigned g1 = (unsigned)((n + 255) / 256);
    k_light_pad<<<g1, 256, 0, st>>>(ipe, L->xp.p, L->Kp, L->Ks, T, nd);
    const dim3 gt((unsigned)((T + kLScintTicks - 1) / kLScintTicks), (unsigned)nd);
    k_light_scint<<<gt, kLWG, 0, st>>>(L->xp.p, L->Kp, L->Ks, T, L->w.p, L->nkb, mu_d);
    k_light_fluct<<<g1, 256, 0, st>>>(mu_d, pe_d, L->pef.p, L->Rp, T, nd, event_id, L->k0, L->k1, q.normal_above);
    if (L->F > 0) {
        const int64_t nc = (int64_t)nd * L->F;
        k_light_noise_coef<<<(unsigned)((nc + 255) / 256), 256, 0, st>>>(L->amp.p, L->F, nd, event_id, L->k0, L->k1,
                                                                        L->coef.p);
    }
    const float *nzpre = nullptr;
    if (L->F > 0 && L->fft_log2 > 0) {
        k_light_noise_fft<<<(unsigned)nd, 1024, noise_fft_lds((size_t)T), st>>>(L->coef.p, L->F, T, L->fft_log2,
                                                                              L->Ct.p, L->nz.p);
        nzpre = L->nz.p;
    }
    const dim3 gr((unsigned)((T + kLTile - 1) / kLTile), (unsigned)nd);
    k_light_response<<<gr, kLWG, 0, st>>>(L->pef.p, L->Rp, T, L->r.p, L->nrb, (float)q.gain, L->coef.p, L->F,
                                         L->Ct.p, L->St.p, nzpre, V);
    if (trig) {
        const int32_t ng = nd / q.group;
        const dim3 gm((unsigned)((T + 255) / 256), (unsigned)ng);
        k_light_trigger_masks<<<gm, 256, 0, st>>>(V, T, q.group, (float)q.trig_threshold, L->tmask.p);
        const size_t lds = sizeof(uint64_t) * (size_t)((T + 63) / 64);
        k_light_trigger_scan<<<(unsigned)ng, 256, lds, st>>>(L->tmask.p, T, q.trig_deadtime, q.max_trig, trig,
                                                             trig_count);
    }
}

void free_graph(lts_light *L) {
    for (int i = 0; i < 2; ++i) {
        if (L->launched[i]) (void)hipEventSynchronize(L->done[i]);
        if (L->exec[i]) (void)hipGraphExecDestroy(L->exec[i]);
        L->exec[i] = nullptr;
        L->launched[i] = false;
    }
    if (L->graph) (void)hipGraphDestroy(L->graph);
    L->graph = nullptr;
    L->fluct_node = L->coef_node = nullptr;
}

// Capture the sequence for these buffers on the simulator's own stream and find the two event-keyed nodes.
lts_status capture_light(lts_light *L, const float *ipe, double *mu_d, double *pe_d, float *V, int32_t *trig,
                         int32_t *trig_count) {
    free_graph(L);
    if (!L->cap_stream) LHIP(L, hipStreamCreateWithFlags(&L->cap_stream, hipStreamNonBlocking));
    LHIP(L, hipStreamBeginCapture(L->cap_stream, hipStreamCaptureModeThreadLocal));
    launch_light(L, 0, ipe, mu_d, pe_d, V, trig, trig_count, L->cap_stream);
    hipGraph_t g = nullptr;
    LHIP(L, hipStreamEndCapture(L->cap_stream, &g));
    L->graph = g;
    size_t nn = 0;
    LHIP(L, hipGraphGetNodes(g, nullptr, &nn));
    std::vector<hipGraphNode_t> nodes(nn);
    LHIP(L, hipGraphGetNodes(g, nodes.data(), &nn));
    for (hipGraphNode_t nd : nodes) {
        hipGraphNodeType ty;
        LHIP(L, hipGraphNodeGetType(nd, &ty));
        if (ty != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams kp;
        LHIP(L, hipGraphKernelNodeGetParams(nd, &kp));
        if (kp.func == reinterpret_cast<void *>(k_light_fluct)) L->fluct_node = nd;
        if (kp.func == reinterpret_cast<void *>(k_light_noise_coef)) L->coef_node = nd;
    }
    if (!L->fluct_node || (L->F > 0 && !L->coef_node))
        return lfail(L, LTS_ERR_DEVICE, "graph capture: event-keyed kernel nodes not found");
    for (int i = 0; i < 2; ++i) {
        LHIP(L, hipGraphInstantiate(&L->exec[i], g, nullptr, nullptr, 0));
        if (!L->done[i]) LHIP(L, hipEventCreateWithFlags(&L->done[i], hipEventDisableTiming));
    }
    return LTS_OK;
}

// Point the two random-number kernel nodes of the instantiated graph at this event.
lts_status set_event(lts_light *L, hipGraphExec_t exec, uint64_t event_id, double *mu_d, double *pe_d) {
    const lts_light_params &q = L->p;
    int32_t T = q.n_ticks, nd = q.n_det, Rp = L->Rp, F = L->F;
    uint32_t k0 = L->k0, k1 = L->k1;
    double na = q.normal_above;
    const double *mu_c = mu_d;
    float *pef = L->pef.p;
    hipKernelNodeParams kp;
    LHIP(L, hipGraphKernelNodeGetParams(L->fluct_node, &kp));
    void *fa[] = {&mu_c, &pe_d, &pef, &Rp, &T, &nd, &event_id, &k0, &k1, &na};
    kp.kernelParams = fa;
    kp.extra = nullptr;
    LHIP(L, hipGraphExecKernelNodeSetParams(exec, L->fluct_node, &kp));
    if (F > 0) {
        const float *amp = L->amp.p;
        float2 *coef = L->coef.p;
        LHIP(L, hipGraphKernelNodeGetParams(L->coef_node, &kp));
        void *ca[] = {&amp, &F, &nd, &event_id, &k0, &k1, &coef};
        kp.kernelParams = ca;
        kp.extra = nullptr;
        LHIP(L, hipGraphExecKernelNodeSetParams(exec, L->coef_node, &kp));
    }
    return LTS_OK;
}

}  // namespace

extern "C" {

lts_status lts_light_create(int device, const lts_light_params *p, const float *resp, int32_t n_resp,
                            const float *noise_amp, int32_t n_freq, lts_light **out) {
    LTS_API_BEGIN
    if (!out) return LTS_ERR_INVALID_ARG;
    *out = nullptr;
    if (!p || !resp || n_resp < 1 || n_resp > (1 << 16) || (n_freq > 0 && !noise_amp) || n_freq < 0)
        return LTS_ERR_INVALID_ARG;
    const lts_light_params &q = *p;
    if (!(q.tick > 0 && q.tau_p > 0 && q.tau_s > 0 && q.f_prompt >= 0 && q.f_prompt <= 1 && q.trunc > 0 &&
          std::isfinite(q.gain) && std::isfinite(q.normal_above) && q.normal_above >= 0 && q.n_det >= 1 &&
          q.n_ticks >= 1 && q.n_ticks <= (1 << 19) && q.group >= 1 && q.n_det % q.group == 0 &&
          std::isfinite(q.trig_threshold) && q.trig_deadtime >= 1 && q.max_trig >= 0 && n_freq < q.n_ticks / 2))
        return LTS_ERR_INVALID_ARG;
    const double kd = std::floor(q.trunc * q.tau_s / q.tick) + 1.0;
    if (!(kd >= 1.0 && kd <= (double)(1 << 22))) return LTS_ERR_INVALID_ARG;
    std::unique_ptr<lts_light> held(new lts_light());   // freed on every failure, exceptions included
    lts_light *L = held.get();
    L->p = q;
    L->device = device;
    L->K = (int32_t)kd;
    L->nkb = (L->K + 7) / 8;
    L->Kp = 8 * L->nkb + 8;
    L->Ks = L->Kp + (q.n_ticks + 7) / 8 * 8;              // row stride: rows start 32-byte aligned
    L->R = n_resp;
    L->nrb = (n_resp + 7) / 8;
    L->Rp = 8 * L->nrb + 8;
    L->F = n_freq;
    L->k0 = (uint32_t)q.seed;
    L->k1 = (uint32_t)(q.seed >> 32);
    auto fin = [&](lts_status s) {
        if (s == LTS_OK) *out = held.release();
        return s;
    };
    if (hipSetDevice(device) != hipSuccess) return fin(LTS_ERR_DEVICE);
    const size_t nd = (size_t)q.n_det, T = (size_t)q.n_ticks;
    // scintillation kernel, sampled two-exponential profile (Sec. 4.2), zero past the truncation
    host_alloc_point();
    std::vector<double> w(8 * (size_t)L->nkb, 0.0);
    for (int32_t k = 0; k < L->K; ++k) {
        const double t = k * q.tick;
        w[k] = q.tick * (q.f_prompt / q.tau_p * std::exp(-t / q.tau_p) + (1.0 - q.f_prompt) / q.tau_s * std::exp(-t / q.tau_s));
    }
    std::vector<float> r(8 * (size_t)L->nrb, 0.0f);
    std::copy(resp, resp + n_resp, r.begin());
    std::vector<float> C(T), S(T);
    for (size_t m = 0; m < T; ++m) {
        const double a = 6.283185307179586477 * (double)m / (double)T;
        C[m] = (float)std::cos(a);
        S[m] = (float)std::sin(a);
    }
    lts_status st = LTS_OK;
    auto ok = [&](hipError_t e) {
        if (e != hipSuccess && st == LTS_OK) st = e == hipErrorOutOfMemory ? LTS_ERR_OOM : LTS_ERR_DEVICE;
        return e == hipSuccess;
    };
    ok(L->w.alloc(w.size())) && ok(L->mu.alloc(nd * T)) && ok(L->pe.alloc(nd * T)) &&
        ok(L->xp.alloc(nd * L->Ks + 16)) && ok(L->pef.alloc(nd * (L->Rp + T) + 8)) && ok(L->r.alloc(r.size())) &&
        ok(L->amp.alloc(std::max(n_freq, 1))) && ok(L->Ct.alloc(T)) && ok(L->St.alloc(T)) &&
        ok(L->coef.alloc(nd * std::max(n_freq, 1))) &&
        ok(L->tmask.alloc(nd / std::max(q.group, 1) * ((T + 63) / 64))) &&
        ok(hipMemcpy(L->w.p, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice)) &&
        ok(hipMemcpy(L->r.p, r.data(), sizeof(float) * r.size(), hipMemcpyHostToDevice)) &&
        (n_freq == 0 || ok(hipMemcpy(L->amp.p, noise_amp, sizeof(float) * n_freq, hipMemcpyHostToDevice))) &&
        ok(hipMemcpy(L->Ct.p, C.data(), sizeof(float) * T, hipMemcpyHostToDevice)) &&
        ok(hipMemcpy(L->St.p, S.data(), sizeof(float) * T, hipMemcpyHostToDevice)) &&
        ok(hipMemset(L->xp.p, 0, sizeof(float) * (nd * L->Ks + 16))) &&
        ok(hipMemset(L->pef.p, 0, sizeof(float) * (nd * (L->Rp + T) + 8))) && ok(hipDeviceSynchronize());
    // power-of-two windows up to 16384 ticks take the FFT noise path if the device grants the LDS it needs
    if (st == LTS_OK && n_freq > 0 && T >= 4 && (T & (T - 1)) == 0 && noise_fft_lds(T) <= 160 * 1024) {
        if (hipFuncSetAttribute((const void *)k_light_noise_fft, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)noise_fft_lds(T)) == hipSuccess &&
            ok(L->nz.alloc(nd * T))) {
            int32_t lg = 0;
            while ((size_t)1 << lg < T) ++lg;
            L->fft_log2 = lg;
        } else {
            (void)hipGetLastError();
        }
    }
    return fin(st);
    LTS_API_END(nullptr)
}

void lts_light_destroy(lts_light *L) {
    if (!L) return;
    (void)hipSetDevice(L->device);
    (void)hipDeviceSynchronize();
    free_graph(L);
    for (int i = 0; i < 2; ++i)
        if (L->done[i]) (void)hipEventDestroy(L->done[i]);
    if (L->cap_stream) (void)hipStreamDestroy(L->cap_stream);
    delete L;
}

lts_status lts_light_set_graph(lts_light *L, int32_t on) {
    LTS_API_BEGIN
    if (!L) return LTS_ERR_INVALID_ARG;
    if (on != 0 && on != 1) return lfail(L, LTS_ERR_INVALID_ARG, "graph must be 0 or 1");
    L->use_graph = on != 0;
    return LTS_OK;
    LTS_API_END(L)
}

lts_status lts_light_simulate(lts_light *L, uint64_t event_id, const float *ipe, double *mu, double *pe, float *V,
                              int32_t *trig, int32_t *trig_count, void *stream) {
    LTS_API_BEGIN
    if (!L) return LTS_ERR_INVALID_ARG;
    if (L->sticky) return lfail(L, LTS_ERR_DEVICE, "a previous device error: destroy and recreate");
    if (!ipe || !V || (!trig) != (!trig_count)) return lfail(L, LTS_ERR_INVALID_ARG, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    LHIP(L, hipSetDevice(L->device));
    double *mu_d = mu ? mu : L->mu.p;
    double *pe_d = pe ? pe : L->pe.p;
    if (!L->use_graph) {
        launch_light(L, event_id, ipe, mu_d, pe_d, V, trig, trig_count, st);
        LHIP(L, hipGetLastError());
        return LTS_OK;
    }
    const void *ptrs[6] = {ipe, mu_d, pe_d, V, trig, trig_count};
    if (!L->exec[0] || memcmp(ptrs, L->g_ptrs, sizeof(ptrs)) != 0) {
        lts_status r = capture_light(L, ipe, mu_d, pe_d, V, trig, trig_count);
        if (r) return r;
        memcpy(L->g_ptrs, ptrs, sizeof(ptrs));
    }
    const int i = L->turn;
    L->turn ^= 1;
    if (L->launched[i]) LHIP(L, hipEventSynchronize(L->done[i]));
    lts_status r = set_event(L, L->exec[i], event_id, mu_d, pe_d);
    if (r) return r;
    LHIP(L, hipGraphLaunch(L->exec[i], st));
    LHIP(L, hipEventRecord(L->done[i], st));
    L->launched[i] = true;
    return LTS_OK;
    LTS_API_END(L)
}

const char *lts_light_last_error(const lts_light *L) { return L ? L->err.c_str() : "null light simulator"; }

}  // extern "C"
