// Narrowband detection pass over a spectral cube (the paper's Sec. 2.4, Stage I with the
// width-1 matched filter), gfx950.
//
// Per-pixel kernel: a workgroup stages the spectra of PPW neighbouring pixels in LDS (one
// read of the cube), and one wave per pixel computes the exact median and MAD by radix
// selection on order-preserving integer keys of the float32 values (4 digit passes of 8 bits,
// histograms in LDS), then scores every channel and keeps threshold crossings that survive
// +-1 channel non-maximum suppression (ties keep the lower channel).  Candidates are appended
// with a global atomic counter and sorted afterwards by (y, x, c) with a bitonic network.
//
// Per-image mode first computes each channel image's median and MAD over the visible
// hemisphere (radix selection over the image in global memory, one workgroup per channel),
// then runs the per-pixel kernel on the standardised values with only the spectral median
// removed.
#include "internal.h"

namespace {

constexpr float MAD_K = 1.482602218505602f;

__device__ __forceinline__ unsigned fkey(float f) {
    unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float funkey(unsigned u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__device__ __forceinline__ bool in_horizon(int x, int y, int n) {
    const int h = n / 2, dx = x - h, dy = y - h;
    return dx * dx + dy * dy < h * h;
}

__device__ __forceinline__ int wave_inclusive_scan(int v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ unsigned wave_min_u(unsigned v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = min(v, (unsigned)__shfl_xor((int)v, d, 64));
    return v;
}

// Value whose key is the rank-th smallest (0-based) of keyfn(i), i < n, for one wave.
// hist: this wave's 256 LDS counters.  Every wave of the block calls this the same number of
// times, so the block barriers inside are uniform.
template <typename KeyFn>
__device__ unsigned wave_select(KeyFn keyfn, int n, int rank, unsigned *hist, int lane) {
    unsigned prefix = 0, pmask = 0;
    int k = rank;
    for (int shift = 24; shift >= 0; shift -= 8) {
#pragma unroll
        for (int b = 0; b < 4; b++) hist[lane * 4 + b] = 0;
        __syncthreads();
        for (int i = lane; i < n; i += 64) {
            const unsigned key = keyfn(i);
            if ((key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        int cnt[4], s = 0;
#pragma unroll
        for (int b = 0; b < 4; b++) {
            cnt[b] = (int)hist[lane * 4 + b];
            s += cnt[b];
        }
        const int incl = wave_inclusive_scan(s, lane);
        const int excl = incl - s;
        int digit = 0, below = 0;
        const bool mine = (excl <= k) && (k < incl);
        if (mine) {
            int run = excl;
#pragma unroll
            for (int b = 0; b < 4; b++) {
                if (k >= run && k < run + cnt[b]) {
                    digit = lane * 4 + b;
                    below = run;
                }
                run += cnt[b];
            }
        }
        const unsigned long long ball = __ballot(mine);
        const int src = ball ? (int)(__ffsll((long long)ball) - 1) : 0;
        digit = __shfl(digit, src, 64);
        below = __shfl(below, src, 64);
        prefix |= (unsigned)digit << shift;
        pmask |= 0xffu << shift;
        k -= below;
        __syncthreads();
    }
    return prefix;
}

// Median of keyfn over n values (mean of the central pair for even n), as float.
template <typename KeyFn>
__device__ float wave_median(KeyFn keyfn, int n, unsigned *hist, int lane) {
    const unsigned klo = wave_select(keyfn, n, (n - 1) / 2, hist, lane);
    if (n & 1) return funkey(klo);
    // rank n/2: equal to klo when more than n/2 keys are <= klo, else the next larger key
    int le = 0;
    unsigned nxt = 0xffffffffu;
    for (int i = lane; i < n; i += 64) {
        const unsigned key = keyfn(i);
        le += key <= klo;
        if (key > klo) nxt = min(nxt, key);
    }
    le = wave_sum(le);
    nxt = wave_min_u(nxt);
    const unsigned khi = (le >= n / 2 + 1) ? klo : nxt;
    return 0.5f * (funkey(klo) + funkey(khi));
}

// stats: per-channel (median, k * MAD) for PER_IMAGE mode, else unused.
template <int PPW>
__global__ __launch_bounds__(64 * PPW) void detect_pixel_kernel(
    const float *__restrict__ img, int n_chan, int n_pix, int mode, const float2 *__restrict__ stats,
    float thresh, float *__restrict__ snr_out, nbsi_cand *__restrict__ cand, int cap, int *__restrict__ counter,
    int n_groups) {
    extern __shared__ float spec[];  // [PPW][n_chan]
    __shared__ unsigned hist_all[PPW][256];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    // XCD-aware order: consecutive pixel groups of one XCD share cache lines of the cube rows
    const int id = blockIdx.x;
    const int xcd = id & 7, slot = id >> 3;
    const int grp = (slot >> 3) * 64 + xcd * 8 + (slot & 7);
    const size_t npix2 = (size_t)n_pix * n_pix;
    const int groups_per_row = n_pix / PPW;
    const bool grp_ok = grp < n_groups;
    const int gy = grp_ok ? grp / groups_per_row : 0;
    const int gx0 = grp_ok ? (grp % groups_per_row) * PPW : 0;
    // stage PPW consecutive pixels of row gy, all channels
    for (int e = t; e < PPW * n_chan; e += 64 * PPW) {
        const int c = e / PPW, pl = e % PPW;
        float v = 0.f;
        if (grp_ok) {
            v = img[(size_t)c * npix2 + (size_t)gy * n_pix + gx0 + pl];
            if (mode == NBSI_DETECT_PER_IMAGE) {
                const float2 st = stats[c];
                v = st.y > 0.f ? (v - st.x) / st.y : 0.f;
            }
        }
        spec[pl * n_chan + c] = v;
    }
    __syncthreads();
    const int x = gx0 + wave, y = gy;
    const bool active = grp_ok && in_horizon(x, y, n_pix);
    float *s = spec + wave * n_chan;
    unsigned *hist = hist_all[wave];
    auto key_x = [&](int i) { return fkey(s[i]); };
    const float med = wave_median(key_x, n_chan, hist, lane);
    float scale = 1.f;  // SNR = (x - med) / scale
    bool ok = active;
    if (mode == NBSI_DETECT_PER_PIXEL) {
        auto key_d = [&](int i) { return fkey(fabsf(s[i] - med)); };
        const float mad = wave_median(key_d, n_chan, hist, lane);
        scale = MAD_K * mad;
        ok = ok && mad > 0.f;
    }
    if (snr_out && grp_ok) {
        for (int c = lane; c < n_chan; c += 64)
            snr_out[(size_t)c * npix2 + (size_t)y * n_pix + x] = ok ? (s[c] - med) / scale : 0.f;
    }
    if (!ok) return;
    for (int c = lane; c < n_chan; c += 64) {
        const float z = (s[c] - med) / scale;
        if (z < thresh) continue;
        if (c > 0 && !(z > (s[c - 1] - med) / scale)) continue;
        if (c + 1 < n_chan && !(z >= (s[c + 1] - med) / scale)) continue;
        const int idx = atomicAdd(counter, 1);
        if (idx < cap) {
            nbsi_cand r;
            r.x = x;
            r.y = y;
            r.c = c;
            r.width = 1;
            r.snr = z;
            cand[idx] = r;
        }
    }
}

// Per-channel median and k*MAD over the visible hemisphere (PER_IMAGE mode).
__global__ __launch_bounds__(64) void image_stats_kernel(const float *__restrict__ img, int n_pix,
                                                         float2 *__restrict__ stats) {
    __shared__ unsigned hist[256];
    const int c = blockIdx.x, lane = threadIdx.x;
    const float *im = img + (size_t)c * n_pix * n_pix;
    int n_in = 0;
    for (int i = lane; i < n_pix * n_pix; i += 64) n_in += in_horizon(i % n_pix, i / n_pix, n_pix);
    n_in = wave_sum(n_in);
    // scan the full image; pixels outside the hemisphere get the largest key
    const int n_all = n_pix * n_pix;
    auto key_x = [&](int i) -> unsigned {
        const int y = i / n_pix, x = i % n_pix;
        return in_horizon(x, y, n_pix) ? fkey(im[i]) : 0xffffffffu;
    };
    // the n_in smallest keys are exactly the in-horizon pixels
    const unsigned klo = wave_select(key_x, n_all, (n_in - 1) / 2, hist, lane);
    float med;
    {
        int le = 0;
        unsigned nxt = 0xffffffffu;
        for (int i = lane; i < n_all; i += 64) {
            const unsigned key = key_x(i);
            le += key <= klo;
            if (key > klo) nxt = min(nxt, key);
        }
        le = wave_sum(le);
        nxt = wave_min_u(nxt);
        const unsigned khi = (n_in & 1) ? klo : ((le >= n_in / 2 + 1) ? klo : nxt);
        med = 0.5f * (funkey(klo) + funkey(khi));
    }
    auto key_d = [&](int i) -> unsigned {
        const int y = i / n_pix, x = i % n_pix;
        return in_horizon(x, y, n_pix) ? fkey(fabsf(im[i] - med)) : 0xffffffffu;
    };
    const unsigned dlo = wave_select(key_d, n_all, (n_in - 1) / 2, hist, lane);
    float mad;
    {
        int le = 0;
        unsigned nxt = 0xffffffffu;
        for (int i = lane; i < n_all; i += 64) {
            const unsigned key = key_d(i);
            le += key <= dlo;
            if (key > dlo) nxt = min(nxt, key);
        }
        le = wave_sum(le);
        nxt = wave_min_u(nxt);
        const unsigned dhi = (n_in & 1) ? dlo : ((le >= n_in / 2 + 1) ? dlo : nxt);
        mad = 0.5f * (funkey(dlo) + funkey(dhi));
    }
    if (lane == 0) stats[c] = make_float2(med, MAD_K * mad);
}

__device__ __forceinline__ unsigned long long cand_key(const nbsi_cand &r, int n_chan, int n_pix) {
    return ((unsigned long long)((unsigned)r.y * (unsigned)n_pix + (unsigned)r.x)) * (unsigned)n_chan +
           (unsigned)r.c;
}

__global__ void sort_keys_kernel(const nbsi_cand *__restrict__ cand, int n, int n_pow2, int n_chan, int n_pix,
                                 unsigned long long *__restrict__ keys) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pow2) return;
    // key in the high bits, original index in the low 24 bits
    keys[i] = (i < n) ? ((cand_key(cand[i], n_chan, n_pix) << 24) | (unsigned long long)i) : ~0ull;
}

__global__ void bitonic_step_kernel(unsigned long long *__restrict__ keys, int n_pow2, int j, int k) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pow2) return;
    const int p = i ^ j;
    if (p > i) {
        const unsigned long long a = keys[i], b = keys[p];
        const bool up = (i & k) == 0;
        if ((a > b) == up) {
            keys[i] = b;
            keys[p] = a;
        }
    }
}

__global__ void gather_sorted_kernel(const unsigned long long *__restrict__ keys, const nbsi_cand *__restrict__ cand,
                                     int n_out, nbsi_cand *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_out) return;
    out[i] = cand[(int)(keys[i] & 0xffffffull)];
}

}  // namespace

int detect_ppw(int n_chan) {
    int ppw = 65536 / (n_chan * 4);
    if (ppw >= 4) return 4;
    if (ppw >= 2) return 2;
    return 1;
}

hipError_t launch_detect_stats(const float *img, int n_chan, int n_pix, int mode, float *stats,
                               hipStream_t st) {
    if (mode != NBSI_DETECT_PER_IMAGE) return hipSuccess;
    hipLaunchKernelGGL(image_stats_kernel, dim3(n_chan), dim3(64), 0, st, img, n_pix,
                       reinterpret_cast<float2 *>(stats));
    return hipGetLastError();
}

hipError_t launch_detect_scan(const float *img, int n_chan, int n_pix, int mode, const float *stats,
                              float thresh, float *snr, nbsi_cand *cand, int cap, int *counter,
                              hipStream_t st) {
    const int ppw = detect_ppw(n_chan);
    const int n_groups = n_pix * n_pix / ppw;
    // grid covers every group id produced by the XCD-aware mapping (blocks of 64 groups)
    const int n_blocks = ((n_groups + 63) / 64) * 64;
    const size_t lds = (size_t)ppw * n_chan * sizeof(float);
    const float2 *s2 = reinterpret_cast<const float2 *>(stats);
    // the staged spectra may exceed the default 64 KiB of dynamic LDS (gfx950 has 160 KiB)
    hipError_t ea = hipSuccess;
    if (ppw == 4) ea = hipFuncSetAttribute((const void *)detect_pixel_kernel<4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    else if (ppw == 2) ea = hipFuncSetAttribute((const void *)detect_pixel_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    else ea = hipFuncSetAttribute((const void *)detect_pixel_kernel<1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ea != hipSuccess) return ea;
    switch (ppw) {
        case 4:
            hipLaunchKernelGGL(detect_pixel_kernel<4>, dim3(n_blocks), dim3(256), lds, st, img, n_chan, n_pix, mode,
                               s2, thresh, snr, cand, cap, counter, n_groups);
            break;
        case 2:
            hipLaunchKernelGGL(detect_pixel_kernel<2>, dim3(n_blocks), dim3(128), lds, st, img, n_chan, n_pix, mode,
                               s2, thresh, snr, cand, cap, counter, n_groups);
            break;
        default:
            hipLaunchKernelGGL(detect_pixel_kernel<1>, dim3(n_blocks), dim3(64), lds, st, img, n_chan, n_pix, mode,
                               s2, thresh, snr, cand, cap, counter, n_groups);
    }
    return hipGetLastError();
}

hipError_t launch_detect_sort(nbsi_cand *cand, int n, unsigned long long *keys, int n_chan, int n_pix,
                              nbsi_cand *out, int n_out, hipStream_t st) {
    if (n <= 0 || n_out <= 0) return hipSuccess;
    int n_pow2 = 1;
    while (n_pow2 < n) n_pow2 <<= 1;
    const int blocks = (n_pow2 + 255) / 256;
    hipLaunchKernelGGL(sort_keys_kernel, dim3(blocks), dim3(256), 0, st, cand, n, n_pow2, n_chan, n_pix, keys);
    for (int k = 2; k <= n_pow2; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1)
            hipLaunchKernelGGL(bitonic_step_kernel, dim3(blocks), dim3(256), 0, st, keys, n_pow2, j, k);
    hipLaunchKernelGGL(gather_sorted_kernel, dim3((n_out + 255) / 256), dim3(256), 0, st, keys, cand, n_out, out);
    return hipGetLastError();
}
