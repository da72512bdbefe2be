// Full Stage I search (Sec. 2.4): matched filtering of every pixel's spectrum with a bank of
// unit-variance boxcars (the window sum over its noise standard deviation: sqrt(w) for white
// noise, sqrt(w + 2 sum_l (w - l) rho_l) when the caller gives the noise's channel correlations
// rho_l, e.g. those the periodic Hann window puts into imaged cubes), the best SNR and width per
// voxel, a Benjamini-Hochberg threshold over all searched voxels, width-aware non-maximum
// suppression along frequency and a local re-evaluation of every survivor against its flanks.
//
// Kernels:
//  * search_bank_kernel: a workgroup takes 64 consecutive pixels (one per lane) and 128
//    channels (32 per wave).  Each wave loads a quarter of those channels plus the widest
//    window's halo (64 below, 63 above) into registers with coalesced 256-byte row loads, all in
//    flight at once, scans them there and writes exclusive prefix sums along frequency to LDS
//    once (relative to the staged block, so window sums never carry the rounding of a long
//    running sum); for every channel it takes the maximum of (P[s + w] - P[s]) / sigma_w over
//    the widths whose window fits in the band (a test skipped for channels at least 64 from
//    both band edges, where every window fits).  It writes the
//    best SNR and width cubes and adds the in-horizon SNRs at or above a floor F to a histogram
//    (1/32 bins; LDS first, then one global atomic per non-empty bin).  Benjamini-Hochberg never
//    accepts a p-value above q (k q / m <= q), so no voxel with S < Q^-1(q) is ever accepted; F
//    lies at least one bin below Q^-1(q), and the step-up search over the histogram is the
//    search over all m voxels.
//  * The host walks the histogram from the lowest bin up to find the largest k with
//    p_(k) <= k q / m; only a bin where that is undecided by its edges is gathered exactly
//    (search_gather_kernel) and sorted on the host.
//  * search_accept_kernel lists the accepted voxels, search_nms_kernel (a thread each) keeps
//    those no neighbour suppresses, and search_refine_kernel (a workgroup per survivor)
//    re-evaluates them, its medians from an exact rank count over at most 512 flank values.
#include "internal.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

namespace {

constexpr int SB_PX = 64;                                    // pixels per workgroup
constexpr int SB_CB = 128;                                   // channels per workgroup
constexpr int SB_HALO_L = NBSI_SEARCH_MAX_WIDTH / 2;         // floor(w / 2) <= 64
constexpr int SB_HALO_R = NBSI_SEARCH_MAX_WIDTH / 2 - 1;     // w - floor(w / 2) - 1 <= 63
constexpr int SB_ROWS = SB_CB + SB_HALO_L + SB_HALO_R;       // staged channels
constexpr int HIST_PER_UNIT = 32;
constexpr int HIST_SPAN = 64;                                // SNR units of 1/32 bins above F
constexpr int HIST_BINS = HIST_SPAN * HIST_PER_UNIT + 1;     // [F, F + 64) in 1/32 steps, then >= F + 64
constexpr int FLANK_MAX = 4 * NBSI_SEARCH_MAX_WIDTH;         // two flanks of at most 2 w_max each
constexpr int REEVAL_MIN_FLANK = 8;
constexpr float MAD_TO_SIGMA = 1.482602218505602f;

// The width bank: widths ascending, and per width the standard deviation sigma_w of the window
// sum of unit-variance noise with the caller's channel correlations (sqrt(w) when white) and its
// reciprocal.
struct Widths {
    int n;
    int w[NBSI_SEARCH_MAX_WIDTHS];
    float inv_sqrt[NBSI_SEARCH_MAX_WIDTHS];  // 1 / sigma_w
    float sigma[NBSI_SEARCH_MAX_WIDTHS];     // sigma_w
};

struct Cand {  // an accepted voxel
    int c, p, w;
    float s;
};

__device__ __forceinline__ bool in_horizon(int p, int n_pix) {
    const int y = p / n_pix, x = p - y * n_pix, h = n_pix / 2;
    return (x - h) * (x - h) + (y - h) * (y - h) < h * h;
}

// Bin of an SNR s >= F = f32 / 32: bin j holds [(f32 + j) / 32, (f32 + j + 1) / 32).  s * 32 is
// exact (a power-of-two scale), so the bin edges are exact and no value lands beside its bin.
__device__ __forceinline__ int hist_bin(float s, int f32) {
    const float u = s * (float)HIST_PER_UNIT;
    return u >= (float)(f32 + HIST_BINS - 1) ? HIST_BINS - 1 : (int)floorf(u) - f32;
}

// Order-preserving map of a float to an unsigned key (negative values below positive ones).
__device__ __forceinline__ unsigned order_key(float s) {
    const unsigned b = __float_as_uint(s);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__global__ __launch_bounds__(256) void search_bank_kernel(const float *__restrict__ r, int n_chan, int n_pix,
                                                          Widths W, int f32, float *__restrict__ best,
                                                          uint8_t *__restrict__ wbest, unsigned *__restrict__ hist) {
    __shared__ float P[(SB_ROWS + 1) * SB_PX];  // P[i][lane] = sum of staged rows < i (exclusive)
    __shared__ float seg_tot[4][SB_PX];
    __shared__ unsigned h_lds[HIST_BINS];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int npx = n_pix * n_pix;
    const int p0 = blockIdx.x * SB_PX, c0 = blockIdx.y * SB_CB;
    const int base = c0 - SB_HALO_L;  // channel of staged row 0
    for (int i = t; i < HIST_BINS; i += 256) h_lds[i] = 0u;
    // wave w loads its own segment of staged rows (one 256-byte row per load, its lane's pixel)
    // into registers, all loads in flight at once, scans it there and writes the prefix sums
    // once, offset by the totals of the segments below (rows outside the band or past the last
    // pixel are zero)
    constexpr int SEG = (SB_ROWS + 3) / 4;
    const int i0 = wave * SEG, i1 = min(SB_ROWS, i0 + SEG);
    const int pp = p0 + lane;
    float v[SEG];
#pragma unroll
    for (int k = 0; k < SEG; k++) {
        const int i = i0 + k, ch = base + i;
        v[k] = (i < i1 && ch >= 0 && ch < n_chan && pp < npx) ? r[(size_t)ch * npx + pp] : 0.f;
    }
    float run = 0.f;
#pragma unroll
    for (int k = 0; k < SEG; k++) {
        run += v[k];
        v[k] = run;
    }
    seg_tot[wave][lane] = run;
    if (t < SB_PX) P[t] = 0.f;
    __syncthreads();
    float off = 0.f;
    for (int k = 0; k < wave; k++) off += seg_tot[k][lane];
#pragma unroll
    for (int k = 0; k < SEG; k++)
        if (i0 + k < i1) P[(i0 + k + 1) * SB_PX + lane] = v[k] + off;
    __syncthreads();
    const int p = p0 + lane;
    const float hist_lo = (float)f32 / (float)HIST_PER_UNIT;  // exact
    const bool pix_ok = p < npx;
    const bool hor = pix_ok && in_horizon(p, n_pix);
    // eight channels at a time: sixteen independent LDS reads per width.  Every index stays
    // inside the staged block whether or not the window fits the band (h <= 64, w - h <= 64), so
    // the reads are unconditional and the band test only masks the result.
    constexpr int CQ = 8;
    for (int j = 0; j < SB_CB / 4; j += CQ) {
        const int cb = c0 + wave * (SB_CB / 4) + j;
        if (cb >= n_chan) break;
        float bs[CQ];
        int bw[CQ];
#pragma unroll
        for (int q = 0; q < CQ; q++) {
            bs[q] = -INFINITY;
            bw[q] = 0;
        }
        // every window of these channels fits the band (h <= 64, w - h <= 64): no band test
        const bool interior = cb >= SB_HALO_L && cb + CQ + SB_HALO_L <= n_chan;
        if (interior) {
            for (int k = 0; k < W.n; k++) {  // widths ascending: the narrower one wins ties
                const int w = W.w[k], h = w >> 1;
                const float inv = W.inv_sqrt[k];
                float v[CQ];
#pragma unroll
                for (int q = 0; q < CQ; q++) {
                    const int is = cb + q - base - h;
                    v[q] = (P[(is + w) * SB_PX + lane] - P[is * SB_PX + lane]) * inv;
                }
#pragma unroll
                for (int q = 0; q < CQ; q++) {
                    if (v[q] > bs[q]) {
                        bs[q] = v[q];
                        bw[q] = w;
                    }
                }
            }
        } else {
            for (int k = 0; k < W.n; k++) {
                const int w = W.w[k], h = w >> 1;
                const float inv = W.inv_sqrt[k];
                float v[CQ];
#pragma unroll
                for (int q = 0; q < CQ; q++) {
                    const int is = cb + q - base - h;
                    v[q] = (P[(is + w) * SB_PX + lane] - P[is * SB_PX + lane]) * inv;
                }
#pragma unroll
                for (int q = 0; q < CQ; q++) {
                    const int c = cb + q;
                    const bool fits = c < n_chan && c - h >= 0 && c - h + w <= n_chan;
                    if (fits && v[q] > bs[q]) {
                        bs[q] = v[q];
                        bw[q] = w;
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < CQ; q++) {
            const int c = cb + q;
            if (c >= n_chan) break;
            if (pix_ok) {
                best[(size_t)c * npx + p] = bs[q];
                wbest[(size_t)c * npx + p] = (uint8_t)bw[q];
            }
            if (hor && bs[q] >= hist_lo) atomicAdd(&h_lds[hist_bin(bs[q], f32)], 1u);
        }
    }
    __syncthreads();
    for (int i = t; i < HIST_BINS; i += 256)
        if (h_lds[i]) atomicAdd(&hist[i], h_lds[i]);
}

// SNRs of in-horizon voxels in [lo, hi) (at most cap are written; counter counts all).
__global__ __launch_bounds__(256) void search_gather_kernel(const float *__restrict__ best, int n_chan, int n_pix,
                                                            float lo, float hi, float *__restrict__ vals, int cap,
                                                            int *__restrict__ counter) {
    const int npx = n_pix * n_pix;
    const size_t n = (size_t)n_chan * npx;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
        const float s = best[e];
        if (s >= lo && s < hi && in_horizon((int)(e % npx), n_pix)) {
            const int i = atomicAdd(counter, 1);
            if (i < cap) vals[i] = s;
        }
    }
}

// In-horizon voxels with SNR >= thr (the provisional detections) and the order key of the
// smallest such SNR.
__global__ __launch_bounds__(256) void search_accept_kernel(const float *__restrict__ best,
                                                            const uint8_t *__restrict__ wbest, int n_chan, int n_pix,
                                                            float thr, Cand *__restrict__ out, int cap,
                                                            int *__restrict__ counter, unsigned *__restrict__ min_bits) {
    const int npx = n_pix * n_pix;
    const size_t n = (size_t)n_chan * npx;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
        const float s = best[e];
        if (s >= thr && in_horizon((int)(e % npx), n_pix)) {
            const int i = atomicAdd(counter, 1);
            if (i < cap) out[i] = Cand{(int)(e / npx), (int)(e % npx), (int)wbest[e], s};
            atomicMin(min_bits, order_key(s));
        }
    }
}

// Suppression, one thread per provisional detection: it survives when no other provisional
// detection (SNR >= thr) at its pixel within max(floor(w/2), 1) channels is higher (below: or
// equal, the lower channel winning ties); survivors are appended to surv.
__global__ __launch_bounds__(256) void search_nms_kernel(const float *__restrict__ best, int n_chan, int n_pix,
                                                         const Cand *__restrict__ cands, int n, float thr,
                                                         Cand *__restrict__ surv, int *__restrict__ counter) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const Cand cd = cands[i];
    const size_t npx = (size_t)n_pix * n_pix;
    const int h = max(cd.w >> 1, 1);
    bool beaten = false;
    for (int d = 1; d <= h && !beaten; d++) {  // nearest neighbours first
        if (cd.c - d >= 0) {
            const float o = best[(size_t)(cd.c - d) * npx + cd.p];
            beaten = o >= thr && o >= cd.s;
        }
        if (!beaten && cd.c + d < n_chan) {
            const float o = best[(size_t)(cd.c + d) * npx + cd.p];
            beaten = o >= thr && o > cd.s;
        }
    }
    if (!beaten) surv[atomicAdd(counter, 1)] = cd;
}

// Exact order statistic of rank k among vals[0..n) in LDS (ties broken by index), by counting.
__device__ float rank_value(const float *vals, int n, int k, float *slot) {
    const int t = threadIdx.x;
    for (int i = t; i < n; i += 256) {
        const float v = vals[i];
        int rank = 0;
        for (int j = 0; j < n; j++) {
            const float u = vals[j];
            rank += (u < v || (u == v && j < i)) ? 1 : 0;
        }
        if (rank == k) *slot = v;
    }
    __syncthreads();
    const float out = *slot;
    __syncthreads();
    return out;
}

__device__ float median_lds(const float *vals, int n, float *slot) {
    const float a = rank_value(vals, n, (n - 1) / 2, slot);
    const float b = rank_value(vals, n, n / 2, slot);
    return 0.5f * (a + b);
}

// One workgroup per survivor of the suppression: keep[i] = its SNR re-evaluated against its
// flanks reproduces at or above S*.
__global__ __launch_bounds__(256) void search_refine_kernel(const float *__restrict__ r, int n_chan, int n_pix,
                                                            const Cand *__restrict__ cands, float sstar,
                                                            Widths W, int *__restrict__ keep) {
    __shared__ float flank[FLANK_MAX];
    __shared__ float dev[FLANK_MAX];
    __shared__ float red[256];
    __shared__ float slot;
    const int t = threadIdx.x;
    const Cand cd = cands[blockIdx.x];
    const int npx = n_pix * n_pix;
    // re-evaluation against the flanks outside a guard of w channels on each side
    const int w = cd.w, s0 = cd.c - (w >> 1), g = w, L = max(16, 2 * w);
    const int la = max(0, s0 - g - L), lb = max(0, s0 - g);              // left flank [la, lb)
    const int ra = min(n_chan, s0 + w + g), rb = min(n_chan, s0 + w + g + L);  // right [ra, rb)
    const int nl = max(0, lb - la), nr = max(0, rb - ra), n = nl + nr;
    if (n < REEVAL_MIN_FLANK) {
        if (t == 0) keep[blockIdx.x] = 0;
        return;
    }
    for (int i = t; i < n; i += 256) {
        const int ch = i < nl ? la + i : ra + (i - nl);
        flank[i] = r[(size_t)ch * npx + cd.p];
    }
    __syncthreads();
    const float b = median_lds(flank, n, &slot);
    for (int i = t; i < n; i += 256) dev[i] = fabsf(flank[i] - b);
    __syncthreads();
    const float mad = median_lds(dev, n, &slot);
    float part = 0.f;
    for (int j = t; j < w; j += 256) part += r[(size_t)(s0 + j) * npx + cd.p] - b;
    red[t] = part;
    __syncthreads();
    for (int sdn = 128; sdn > 0; sdn >>= 1) {
        if (t < sdn) red[t] += red[t + sdn];
        __syncthreads();
    }
    if (t == 0) {
        const float sigma = MAD_TO_SIGMA * mad;
        float sw = sqrtf((float)w);  // (every candidate's width is one of the bank's)
        for (int k = 0; k < W.n; k++)
            if (W.w[k] == w) sw = W.sigma[k];
        const float snr2 = sigma > 0.f ? red[0] / (sw * sigma) : -INFINITY;
        keep[blockIdx.x] = snr2 >= sstar ? 1 : 0;
    }
}

double q_tail(double s) { return 0.5 * erfc(s / sqrt(2.0)); }

}  // namespace

extern "C" int nbsi_search_corr(nbsi_ctx *ctx, const float *snr, int n_chan, int n_pix, const int32_t *widths_host,
                                int n_widths, const double *rho_host, int n_rho, double fdr_q, float *best_snr,
                                uint8_t *best_width, nbsi_cand *out, int max_out, int *n_out, float *thresh_host,
                                int64_t *n_provisional_host) {
    if (!ctx) return NBSI_EINVAL;
    int rc = nbsi_check_detect(n_chan, n_pix, NBSI_DETECT_PER_PIXEL, max_out);
    if (rc) return nbsi_fail(ctx, rc, "nbsi_search: bad shape");
    if (!snr || !n_out || (max_out > 0 && !out)) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_search: null pointer");
    if (!aligned16(snr) || (out && !aligned16(out)) || (best_snr && !aligned16(best_snr)) ||
        (best_width && !aligned16(best_width)))
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_search: misaligned pointer");
    if (!(fdr_q > 0.0 && fdr_q < 1.0)) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_search: fdr_q must be in (0, 1)");
    if (n_rho < 0 || n_rho > NBSI_SEARCH_MAX_LAG || (n_rho > 0 && !rho_host))
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_search: n_rho out of range or rho missing");
    for (int l = 0; l < n_rho; l++)
        if (!(rho_host[l] > -1.0 && rho_host[l] < 1.0))
            return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_search: channel correlations must be in (-1, 1)");
    static const int kDefault[] = {1,  2,  3,  4,  5,  6,  7,  8,  9,  10, 12, 16, 20,
                                   24, 28, 32, 36, 40, 44, 48, 50, 60, 70, 80, 90, 100};
    std::vector<int> ws;
    if (widths_host) {
        if (n_widths < 1 || n_widths > NBSI_SEARCH_MAX_WIDTHS)
            return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_search: n_widths out of range");
        ws.assign(widths_host, widths_host + n_widths);
    } else {
        ws.assign(kDefault, kDefault + sizeof(kDefault) / sizeof(kDefault[0]));
    }
    std::sort(ws.begin(), ws.end());
    ws.erase(std::unique(ws.begin(), ws.end()), ws.end());
    if (ws.front() < 1 || ws.back() > NBSI_SEARCH_MAX_WIDTH)
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_search: widths must be in [1, NBSI_SEARCH_MAX_WIDTH]");
    Widths W{};
    W.n = (int)ws.size();
    for (int k = 0; k < W.n; k++) {
        // variance of the sum of w consecutive unit-variance samples: w + 2 sum_l (w - l) rho_l
        const int w = ws[k];
        double var = (double)w;
        for (int l = 1; l <= std::min(w - 1, n_rho); l++) var += 2.0 * (double)(w - l) * rho_host[l - 1];
        if (!(var > 0.0))
            return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_search: channel correlations give a window sum of no variance");
        W.w[k] = w;
        W.inv_sqrt[k] = (float)(1.0 / sqrt(var));
        W.sigma[k] = (float)sqrt(var);
    }
    // histogram floor F = f32 / 32: a whole bin below Q^-1(q) (q_tail(f32 / 32 + 1 / 32) > q), far
    // beyond erfc's rounding, so every voxel BH can accept is counted
    int kq = -32 * HIST_PER_UNIT;
    while (kq < HIST_SPAN * HIST_PER_UNIT && q_tail((double)(kq + 1) / HIST_PER_UNIT) > fdr_q) kq++;
    const int f32 = kq - 1;
    DeviceGuard g(ctx->device);
    const size_t npx = (size_t)n_pix * n_pix, nvox = (size_t)n_chan * npx;
    void *S = best_snr, *Wc = best_width, *hist = nullptr;
    if (!S && (rc = nbsi_scratch(ctx, SLOT_SEARCH_S, sizeof(float) * nvox, &S))) return rc;
    if (!Wc && (rc = nbsi_scratch(ctx, SLOT_SEARCH_W, nvox, &Wc))) return rc;
    if ((rc = nbsi_scratch(ctx, SLOT_SEARCH_HIST, sizeof(unsigned) * HIST_BINS, &hist))) return rc;
    NBSI_TRY_HIP(ctx, hipMemsetAsync(hist, 0, sizeof(unsigned) * HIST_BINS, ctx->stream));
    hipLaunchKernelGGL(search_bank_kernel, dim3((unsigned)((npx + SB_PX - 1) / SB_PX), (unsigned)((n_chan + SB_CB - 1) / SB_CB)),
                       dim3(256), 0, ctx->stream, snr, n_chan, n_pix, W, f32, (float *)S, (uint8_t *)Wc, (unsigned *)hist);
    NBSI_TRY_HIP(ctx, hipGetLastError());
    std::vector<unsigned> h(HIST_BINS);
    NBSI_TRY_HIP(ctx, hipMemcpyAsync(h.data(), hist, sizeof(unsigned) * HIST_BINS, hipMemcpyDeviceToHost, ctx->stream));
    NBSI_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));

    // number of searched voxels: in-horizon pixels x channels
    int64_t n_hor = 0;
    const int hp = n_pix / 2;
    for (int y = 0; y < n_pix; y++)
        for (int x = 0; x < n_pix; x++) n_hor += ((x - hp) * (x - hp) + (y - hp) * (y - hp) < hp * hp) ? 1 : 0;
    const double m = (double)n_hor * (double)n_chan;
    std::vector<int64_t> above(HIST_BINS + 1, 0);  // above[j] = #{S >= lower edge of bin j}
    for (int j = HIST_BINS - 1; j >= 0; j--) above[j] = above[j + 1] + h[j];
    auto lo_of = [f32](int j) { return (double)(f32 + j) / HIST_PER_UNIT; };

    // Benjamini-Hochberg: the largest k with p_(k) <= k q / m.  Bins are visited from the lowest
    // SNR (largest k) up; a bin is skipped when even its highest SNR cannot satisfy the rule,
    // accepted whole when its lowest edge already does, and otherwise resolved exactly.
    int64_t kstar = 0;
    float thr_acc = INFINITY;  // accept S >= thr_acc
    float sstar = INFINITY;    // the k*-th largest S
    bool exact = false;
    for (int j = 0; j < HIST_BINS && kstar == 0; j++) {
        if (h[j] == 0) continue;
        const int64_t nj = above[j], nj1 = above[j + 1];
        const double lo = lo_of(j), hi = (j == HIST_BINS - 1) ? INFINITY : lo_of(j + 1);
        if (!(q_tail(hi) < (double)nj * fdr_q / m)) continue;
        if (q_tail(lo) <= (double)nj * fdr_q / m) {
            kstar = nj;
            thr_acc = (float)lo;
            break;
        }
        void *vals = nullptr;
        if ((rc = nbsi_scratch(ctx, SLOT_SEARCH_VALS, sizeof(float) * (size_t)h[j], &vals))) return rc;
        NBSI_TRY_HIP(ctx, hipMemsetAsync(ctx->d_counter, 0, sizeof(int), ctx->stream));
        hipLaunchKernelGGL(search_gather_kernel, dim3(4096), dim3(256), 0, ctx->stream, (const float *)S, n_chan, n_pix,
                           (float)lo, j == HIST_BINS - 1 ? INFINITY : (float)hi, (float *)vals, (int)h[j], ctx->d_counter);
        NBSI_TRY_HIP(ctx, hipGetLastError());
        std::vector<float> v(h[j]);
        NBSI_TRY_HIP(ctx, hipMemcpyAsync(v.data(), vals, sizeof(float) * v.size(), hipMemcpyDeviceToHost, ctx->stream));
        NBSI_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
        std::sort(v.begin(), v.end(), std::greater<float>());  // k = nj1 + 1 .. nj
        for (int64_t i = (int64_t)v.size() - 1; i >= 0; i--) {
            const int64_t k = nj1 + i + 1;
            if (q_tail((double)v[i]) <= (double)k * fdr_q / m) {
                kstar = k;
                sstar = v[i];
                thr_acc = v[i];
                exact = true;
                break;
            }
        }
    }
    *n_out = 0;
    if (thresh_host) *thresh_host = INFINITY;
    if (n_provisional_host) *n_provisional_host = kstar;
    if (kstar == 0) return NBSI_OK;

    // provisional detections
    const int j_acc = (int)floor((double)thr_acc * HIST_PER_UNIT) - f32;  // the bin holding thr_acc
    const int cap = (int)above[std::min(HIST_BINS - 1, std::max(0, j_acc))];
    void *cands = nullptr, *keep = nullptr;
    if ((rc = nbsi_scratch(ctx, SLOT_SEARCH_CAND, sizeof(Cand) * (size_t)std::max(cap, 1), &cands))) return rc;
    if ((rc = nbsi_scratch(ctx, SLOT_SEARCH_KEEP, sizeof(int) * (size_t)std::max(cap, 1), &keep))) return rc;
    const unsigned init[2] = {0u, 0xffffffffu};  // counter, the largest order key
    NBSI_TRY_HIP(ctx, hipMemcpyAsync(ctx->d_counter, init, sizeof(init), hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(search_accept_kernel, dim3(4096), dim3(256), 0, ctx->stream, (const float *)S, (const uint8_t *)Wc,
                       n_chan, n_pix, thr_acc, (Cand *)cands, cap, ctx->d_counter, (unsigned *)(ctx->d_counter + 1));
    NBSI_TRY_HIP(ctx, hipGetLastError());
    unsigned got[2] = {0u, 0u};
    NBSI_TRY_HIP(ctx, hipMemcpyAsync(got, ctx->d_counter, sizeof(got), hipMemcpyDeviceToHost, ctx->stream));
    NBSI_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const int n_acc = (int)got[0];
    if (n_acc > cap) return nbsi_fail(ctx, NBSI_EHIP, "nbsi_search: provisional detections exceed the histogram count");
    if (!exact) {  // invert the order key of the smallest accepted SNR
        const unsigned bits = (got[1] & 0x80000000u) ? (got[1] & 0x7fffffffu) : ~got[1];
        float mn;
        memcpy(&mn, &bits, sizeof(float));
        sstar = mn;
    }
    if (thresh_host) *thresh_host = sstar;
    void *surv = nullptr;
    if ((rc = nbsi_scratch(ctx, SLOT_SEARCH_SURV, sizeof(Cand) * (size_t)std::max(n_acc, 1), &surv))) return rc;
    NBSI_TRY_HIP(ctx, hipMemsetAsync(ctx->d_counter, 0, sizeof(int), ctx->stream));
    if (n_acc > 0)
        hipLaunchKernelGGL(search_nms_kernel, dim3((unsigned)((n_acc + 255) / 256)), dim3(256), 0, ctx->stream,
                           (const float *)S, n_chan, n_pix, (const Cand *)cands, n_acc, thr_acc, (Cand *)surv,
                           ctx->d_counter);
    NBSI_TRY_HIP(ctx, hipGetLastError());
    int n_surv = 0;
    NBSI_TRY_HIP(ctx, hipMemcpyAsync(&n_surv, ctx->d_counter, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    NBSI_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (n_surv > 0)
        hipLaunchKernelGGL(search_refine_kernel, dim3((unsigned)n_surv), dim3(256), 0, ctx->stream, snr, n_chan, n_pix,
                           (const Cand *)surv, sstar, W, (int *)keep);
    NBSI_TRY_HIP(ctx, hipGetLastError());
    std::vector<Cand> hc(n_surv);
    std::vector<int> hk(n_surv);
    NBSI_TRY_HIP(ctx, hipMemcpyAsync(hc.data(), surv, sizeof(Cand) * n_surv, hipMemcpyDeviceToHost, ctx->stream));
    NBSI_TRY_HIP(ctx, hipMemcpyAsync(hk.data(), keep, sizeof(int) * n_surv, hipMemcpyDeviceToHost, ctx->stream));
    NBSI_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::vector<nbsi_cand> rec;
    for (int i = 0; i < n_surv; i++)
        if (hk[i]) rec.push_back(nbsi_cand{hc[i].p % n_pix, hc[i].p / n_pix, hc[i].c, hc[i].w, hc[i].s});
    std::sort(rec.begin(), rec.end(), [](const nbsi_cand &a, const nbsi_cand &b) {
        return a.y != b.y ? a.y < b.y : a.x != b.x ? a.x < b.x : a.c < b.c;
    });
    *n_out = (int)rec.size();
    const int n_write = std::min((int)rec.size(), max_out);
    if (n_write > 0) {
        NBSI_TRY_HIP(ctx, hipMemcpyAsync(out, rec.data(), sizeof(nbsi_cand) * n_write, hipMemcpyHostToDevice, ctx->stream));
        NBSI_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    return (int)rec.size() > max_out ? NBSI_ETRUNC : NBSI_OK;
}

extern "C" int nbsi_search(nbsi_ctx *ctx, const float *snr, int n_chan, int n_pix, const int32_t *widths_host,
                           int n_widths, double fdr_q, float *best_snr, uint8_t *best_width, nbsi_cand *out,
                           int max_out, int *n_out, float *thresh_host, int64_t *n_provisional_host) {
    return nbsi_search_corr(ctx, snr, n_chan, n_pix, widths_host, n_widths, nullptr, 0, fdr_q, best_snr, best_width,
                            out, max_out, n_out, thresh_host, n_provisional_host);
}
