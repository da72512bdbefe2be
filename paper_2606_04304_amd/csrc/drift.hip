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
// once per workgroup and reused by all 2D + 1 trials from LDS.
#include "internal.h"

#include <algorithm>
#include <mutex>
#include <vector>

namespace {

constexpr int DD_PX = 32;
constexpr int DD_CB = 64;
constexpr int DD_ROWS = DD_CB + 2 * NBSI_DEDOPPLER_MAX_DRIFT;

__device__ __forceinline__ int drift_shift(int d, int s, int n_sub) {
    if (n_sub <= 1 || d == 0 || s == 0) return 0;
    const int ad = d < 0 ? -d : d;
    const int mag = (2 * ad * s + (n_sub - 1)) / (2 * (n_sub - 1));
    return d > 0 ? mag : -mag;
}

__global__ __launch_bounds__(256) void dedoppler_kernel(const float *__restrict__ r, int n_sub, int n_chan,
                                                        int n_pix, int max_drift, float *__restrict__ best,
                                                        int8_t *__restrict__ drift) {
    extern __shared__ float tile[];  // [n_sub][DD_ROWS][DD_PX]
    // staged-row offset of every (trial, sub-integration): (s DD_ROWS + shift(d, s)) DD_PX, trial k
    // being d = 0, -1, +1, -2, +2, ...
    __shared__ int off[(2 * NBSI_DEDOPPLER_MAX_DRIFT + 1) * NBSI_DEDOPPLER_MAX_SUB];
    const int t = threadIdx.x, lane = t & (DD_PX - 1), grp = t / DD_PX;  // 8 groups of 8 channels
    const int n_trials = 2 * max_drift + 1;
    for (int e = t; e < n_trials * n_sub; e += 256) {
        const int k = e / n_sub, s = e % n_sub;
        const int d = (k == 0) ? 0 : ((k & 1) ? -((k + 1) >> 1) : (k >> 1));
        off[e] = (s * DD_ROWS + drift_shift(d, s, n_sub)) * DD_PX;
    }
    const size_t npx = (size_t)n_pix * n_pix;
    const size_t p0 = (size_t)blockIdx.x * DD_PX;
    const int c0 = blockIdx.y * DD_CB;
    const int base = c0 - NBSI_DEDOPPLER_MAX_DRIFT;
    // eight independent loads in flight per thread before their LDS stores
    const int n_el = n_sub * DD_ROWS * DD_PX;
    for (int e0 = t; e0 < n_el; e0 += 8 * 256) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int e = e0 + 256 * u;
            const int l = e % DD_PX, row = (e / DD_PX) % DD_ROWS, s = e / (DD_PX * DD_ROWS);
            const int ch = base + row;
            const size_t p = p0 + l;
            v[u] = (e < n_el && ch >= 0 && ch < n_chan && p < npx) ? r[((size_t)s * n_chan + ch) * npx + p] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 8; u++)
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
        for (int k = 0; k < n_trials; k++) {  // 0, -1, +1, -2, +2, ...
            const int d = (k == 0) ? 0 : ((k & 1) ? -((k + 1) >> 1) : (k >> 1));
            if (c + d < 0 || c + d >= n_chan) continue;
            float acc = 0.f;
            for (int s = 0; s < n_sub; s++) acc += col[off[k * n_sub + s]];
            const float v = acc * inv;
            if (v > bv) {
                bv = v;
                bd = d;
            }
        }
        best[(size_t)c * npx + p] = bv;
        drift[(size_t)c * npx + p] = (int8_t)bd;
    }
}

// More than 64 KB of dynamic LDS (6 to 8 sub-integrations) needs the kernel's limit raised, once
// per device.
hipError_t dedoppler_lds_prepare() {
    static std::mutex mu;
    static std::vector<int> done;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (std::find(done.begin(), done.end(), dev) != done.end()) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute((const void *)dedoppler_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)(sizeof(float) * NBSI_DEDOPPLER_MAX_SUB * DD_ROWS * DD_PX));
    if (e == hipSuccess) done.push_back(dev);
    return e;
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
    NBSI_TRY_HIP(ctx, dedoppler_lds_prepare());
    hipLaunchKernelGGL(dedoppler_kernel, dim3((unsigned)((npx + DD_PX - 1) / DD_PX), (unsigned)((n_chan + DD_CB - 1) / DD_CB)),
                       dim3(256), lds, ctx->stream, snr_sub, n_sub, n_chan, n_pix, max_drift, best, drift);
    NBSI_TRY_HIP(ctx, hipGetLastError());
    return NBSI_OK;
}
