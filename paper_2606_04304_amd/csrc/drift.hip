// Drift-rate search (the paper's Doppler-drift discussion, Sec. 2): residual cubes of S
// sub-integrations of one dump are summed along drifting tracks, c + shift(d, s) in
// sub-integration s with shift(d, s) = round(d s / (S - 1)) (halves away from zero), for every
// total drift d = -D..D channels, as (1 / sqrt(S)) sum_s r_s[c + shift(d, s)]; per voxel the
// largest sum and its drift are kept (trials in the order 0, -1, +1, -2, ... with a strict
// comparison), where the whole track lies in the band.
//
// dedoppler_kernel: a workgroup takes 32 pixels (one per lane of a half-wave) x 64 channels
// (8 per thread) and stages every sub-integration's channels [c0 - D_MAX, c0 + 64 + D_MAX) of
// those pixels in LDS with coalesced 128-byte row loads, so each input value is read from HBM
// once per workgroup and reused by all 2D + 1 trials from LDS.  All 33 trials are evaluated
// (those beyond the requested drift masked), so each distinct (sub-integration, shift) value is
// read once per channel.  Channels at least D_MAX from both band edges with the full drift range
// requested skip the per-trial band test (every track fits).
#include "internal.h"

#include <algorithm>
#include <mutex>
#include <vector>

namespace {

constexpr int DD_PX = 32;
constexpr int DD_CB = 64;
constexpr int DD_ROWS = DD_CB + 2 * NBSI_DEDOPPLER_MAX_DRIFT;

__host__ __device__ constexpr int drift_shift(int d, int s, int n_sub) {
    if (n_sub <= 1 || d == 0 || s == 0) return 0;
    const int ad = d < 0 ? -d : d;
    const int mag = (2 * ad * s + (n_sub - 1)) / (2 * (n_sub - 1));
    return d > 0 ? mag : -mag;
}

// The sub-integration count is a template parameter, so with the trial loop unrolled every
// track offset (s DD_ROWS + shift(d, s)) DD_PX is an immediate of its LDS read, and reads shared
// by several trials are issued once.
template <int NS>
__global__ __launch_bounds__(256) void dedoppler_kernel(const float *__restrict__ r, int n_chan, int n_pix,
                                                        int max_drift, float *__restrict__ best,
                                                        int8_t *__restrict__ drift) {
    constexpr int n_sub = NS;
    extern __shared__ float tile[];  // [n_sub][DD_ROWS][DD_PX]
    const int t = threadIdx.x, lane = t & (DD_PX - 1), grp = t / DD_PX;  // 8 groups of 8 channels
    const size_t npx = (size_t)n_pix * n_pix;
    const size_t p0 = (size_t)blockIdx.x * DD_PX;
    const int c0 = blockIdx.y * DD_CB;
    const int base = c0 - NBSI_DEDOPPLER_MAX_DRIFT;
    // 24 independent loads in flight per thread before their LDS stores
    const int n_el = n_sub * DD_ROWS * DD_PX;
    for (int e0 = t; e0 < n_el; e0 += 24 * 256) {
        float v[24];
#pragma unroll
        for (int u = 0; u < 24; u++) {
            const int e = e0 + 256 * u;
            const int l = e % DD_PX, row = (e / DD_PX) % DD_ROWS, s = e / (DD_PX * DD_ROWS);
            const int ch = base + row;
            const size_t p = p0 + l;
            v[u] = (e < n_el && ch >= 0 && ch < n_chan && p < npx) ? r[((size_t)s * n_chan + ch) * npx + p] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 24; u++)
            if (e0 + 256 * u < n_el) tile[e0 + 256 * u] = v[u];
    }
    __syncthreads();
    const size_t p = p0 + lane;
    if (p >= npx) return;
    const float inv = rsqrtf((float)n_sub);
    for (int j = 0; j < DD_CB / 8; j++) {
        const int c = c0 + grp * (DD_CB / 8) + j;
        if (c >= n_chan) break;
        const int ic = c - base;
        float bv = -INFINITY;
        int bd = 0;
        const float *col = tile + ic * DD_PX + lane;
        // every trial's track lies in the band and is requested: no per-trial test
        const bool all_ok = max_drift == NBSI_DEDOPPLER_MAX_DRIFT && c >= NBSI_DEDOPPLER_MAX_DRIFT &&
                            c + NBSI_DEDOPPLER_MAX_DRIFT < n_chan;
        if (all_ok) {
#pragma unroll
            for (int k = 0; k < 2 * NBSI_DEDOPPLER_MAX_DRIFT + 1; k++) {  // 0, -1, +1, -2, +2, ...
                const int d = (k == 0) ? 0 : ((k & 1) ? -((k + 1) >> 1) : (k >> 1));
                float acc = 0.f;
#pragma unroll
                for (int s = 0; s < n_sub; s++) acc += col[(s * DD_ROWS + drift_shift(d, s, n_sub)) * DD_PX];
                const float v = acc * inv;
                if (v > bv) {
                    bv = v;
                    bd = d;
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < 2 * NBSI_DEDOPPLER_MAX_DRIFT + 1; k++) {
                const int d = (k == 0) ? 0 : ((k & 1) ? -((k + 1) >> 1) : (k >> 1));
                float acc = 0.f;
#pragma unroll
                for (int s = 0; s < n_sub; s++) acc += col[(s * DD_ROWS + drift_shift(d, s, n_sub)) * DD_PX];
                const float v = acc * inv;
                const bool ok = k < 2 * max_drift + 1 && c + d >= 0 && c + d < n_chan;
                if (ok && v > bv) {
                    bv = v;
                    bd = d;
                }
            }
        }
        best[(size_t)c * npx + p] = bv;
        drift[(size_t)c * npx + p] = (int8_t)bd;
    }
}

// More than 64 KB of dynamic LDS (6 to 8 sub-integrations) needs the kernel's limit raised, once
// per device.
template <int NS>
hipError_t dedoppler_launch(dim3 grid, size_t lds, hipStream_t st, const float *r, int n_chan, int n_pix,
                            int max_drift, float *best, int8_t *drift) {
    static std::mutex mu;
    static std::vector<int> done;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
    {
        std::lock_guard<std::mutex> lock(mu);
        if (std::find(done.begin(), done.end(), dev) == done.end()) {
            const hipError_t e = hipFuncSetAttribute((const void *)dedoppler_kernel<NS>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)(sizeof(float) * NS * DD_ROWS * DD_PX));
            if (e != hipSuccess) return e;
            done.push_back(dev);
        }
    }
    hipLaunchKernelGGL(dedoppler_kernel<NS>, grid, dim3(256), lds, st, r, n_chan, n_pix, max_drift, best, drift);
    return hipGetLastError();
}

}  // namespace

extern "C" int nbsi_dedoppler(nbsi_ctx *ctx, const float *snr_sub, int n_sub, int n_chan, int n_pix, int max_drift,
                              float *best, int8_t *drift) {
    if (!ctx) return NBSI_EINVAL;
    if (n_sub < 1 || n_sub > NBSI_DEDOPPLER_MAX_SUB || max_drift < 0 || max_drift > NBSI_DEDOPPLER_MAX_DRIFT)
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_dedoppler: n_sub or max_drift out of range");
    int rc = nbsi_check_detect(n_chan, n_pix, NBSI_DETECT_PER_PIXEL, 0);
    if (rc) return nbsi_fail(ctx, rc, "nbsi_dedoppler: bad shape");
    if (!snr_sub || !best || !drift) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_dedoppler: null pointer");
    if (!aligned16(snr_sub) || !aligned16(best) || !aligned16(drift))
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_dedoppler: misaligned pointer");
    DeviceGuard g(ctx->device);
    const size_t npx = (size_t)n_pix * n_pix;
    const size_t lds = sizeof(float) * (size_t)n_sub * DD_ROWS * DD_PX;
    const dim3 grid((unsigned)((npx + DD_PX - 1) / DD_PX), (unsigned)((n_chan + DD_CB - 1) / DD_CB));
    hipError_t e = hipErrorInvalidValue;
    switch (n_sub) {
        case 1: e = dedoppler_launch<1>(grid, lds, ctx->stream, snr_sub, n_chan, n_pix, max_drift, best, drift); break;
        case 2: e = dedoppler_launch<2>(grid, lds, ctx->stream, snr_sub, n_chan, n_pix, max_drift, best, drift); break;
        case 3: e = dedoppler_launch<3>(grid, lds, ctx->stream, snr_sub, n_chan, n_pix, max_drift, best, drift); break;
        case 4: e = dedoppler_launch<4>(grid, lds, ctx->stream, snr_sub, n_chan, n_pix, max_drift, best, drift); break;
        case 5: e = dedoppler_launch<5>(grid, lds, ctx->stream, snr_sub, n_chan, n_pix, max_drift, best, drift); break;
        case 6: e = dedoppler_launch<6>(grid, lds, ctx->stream, snr_sub, n_chan, n_pix, max_drift, best, drift); break;
        case 7: e = dedoppler_launch<7>(grid, lds, ctx->stream, snr_sub, n_chan, n_pix, max_drift, best, drift); break;
        case 8: e = dedoppler_launch<8>(grid, lds, ctx->stream, snr_sub, n_chan, n_pix, max_drift, best, drift); break;
    }
    NBSI_TRY_HIP(ctx, e);
    return NBSI_OK;
}
