// Upchannelisation (the paper's Sec. 2.1 FFT over the time samples of each coarse channel),
// periodic Hann window, fftshifted channel selection and int8 requantisation, for gfx950.
//
// Design.  Only a contiguous band of C fine channels is kept out of each N-point spectrum,
// so the transform is evaluated as P = N / M sub-transforms of size M >= C on the
// decimated sequences x[p + P m] (m < M):
//     X[k] = sum_p W_N^{p k} Y_p[k mod M],   Y_p = FFT_M(w x)[p + P m]
// Each sub-transform lives in LDS + registers of one workgroup (M/16 threads, 16 complex
// values per thread, radix-16 Stockham passes), and every thread accumulates the kept outputs
// it owns in registers; nothing of the N-point spectrum ever goes to HBM.  Twiddles and the
// window come from a two-level table of float32 roundings of float64 roots (~1.5 ulp).
//
// The workgroup of input i, spectrum s writes its kept band to a staging array
// [n_in][n_spec][C] (coalesced); a corner-turn kernel then produces the correlator layout
// [C][n_in][2][n_spec].
#include "internal.h"
#include "fft_dev.h"

namespace {

constexpr int E = 16;  // complex values per thread

template <int LOGM>
struct Plan {
    static constexpr int M = 1 << LOGM;
    static constexpr int NT = M / E;
    static constexpr int R0 = (LOGM % 4 == 0) ? 16 : (1 << (LOGM % 4));  // first radix
    static constexpr int NPASS16 = (LOGM % 4 == 0) ? LOGM / 4 - 1 : LOGM / 4;
};

template <int LOGM>
__global__ __launch_bounds__((1 << LOGM) / 16) void channelize_kernel(
    const int8_t *__restrict__ volt, int log_n, int n_spec, int klo, int n_chan,
    const float *__restrict__ gain, int8_t *__restrict__ stage_q, float2 *__restrict__ stage_f) {
    using PL = Plan<LOGM>;
    constexpr int M = PL::M, NT = PL::NT, R0 = PL::R0;
    __shared__ float2 buf[M];
    __shared__ float2 tw_lo[512], tw_hi[512];

    const int t = threadIdx.x;
    const int s = blockIdx.x % n_spec;
    const int i = blockIdx.x / n_spec;
    const int N = 1 << log_n;
    const int P = N >> LOGM;
    const int log_p = log_n - LOGM;

    const TwiddleTable tw = build_twiddles(tw_lo, tw_hi, log_n, t, NT);
    __syncthreads();

    const int16_t *x = reinterpret_cast<const int16_t *>(volt) + ((size_t)i * n_spec + s) * (size_t)N;

    // kept outputs owned by this thread: register e = r (final radix-16 pass) holds k1 = t + r*NT
    int kfull[E];
    bool kept[E];
#pragma unroll
    for (int r = 0; r < E; r++) {
        const int k1 = t + r * NT;
        const int d = (k1 - klo) & (M - 1);
        kept[r] = d < n_chan;
        kfull[r] = (klo + d) & (N - 1);
    }

    float2 acc[E];
#pragma unroll
    for (int r = 0; r < E; r++) acc[r] = make_float2(0.f, 0.f);

    for (int p = 0; p < P; p++) {
        float2 v[E];
        // first pass inputs: element m = j + r*M/R0, j = t + NT*b; sample n = p + P*m
#pragma unroll
        for (int b = 0; b < E / R0; b++) {
#pragma unroll
            for (int r = 0; r < R0; r++) {
                const int m = t + NT * b + r * (M / R0);
                const int n = p + (m << log_p);
                const int16_t raw = x[n];
                const float w = 0.5f - 0.5f * tw(n).x;   // periodic Hann: cos(2 pi n / N)
                v[b * R0 + r] = make_float2(w * (float)(int8_t)(raw & 0xff), w * (float)(int8_t)(raw >> 8));
            }
        }
        stockham_regs<R0, E>(v, t, NT, LOGM, 1, tw, log_n);
        int ns = R0;
        if constexpr (PL::NPASS16 > 0) {
            __syncthreads();  // buf free (previous sub-transform done reading)
            stockham_store<R0, E>(buf, v, t, NT, 1);
            __syncthreads();
#pragma unroll
            for (int pass = 0; pass < PL::NPASS16; pass++) {
                stockham_load<16, E>(buf, v, t, NT, LOGM);
                stockham_regs<16, E>(v, t, NT, LOGM, ns, tw, log_n);
                if (pass + 1 < PL::NPASS16) {
                    __syncthreads();
                    stockham_store<16, E>(buf, v, t, NT, ns);
                    __syncthreads();
                }
                ns *= 16;
            }
        }
        // v[r] = Y_p[t + r*NT]
        if (P == 1) {
#pragma unroll
            for (int r = 0; r < E; r++) acc[r] = v[r];
        } else {
#pragma unroll
            for (int r = 0; r < E; r++) {
                if (kept[r]) acc[r] = cadd(acc[r], cmul(v[r], tw((p * kfull[r]) & (N - 1))));
            }
        }
    }

    const float g = gain[i];
    const size_t row = ((size_t)i * n_spec + s) * (size_t)n_chan;
#pragma unroll
    for (int r = 0; r < E; r++) {
        if (!kept[r]) continue;
        const int k1 = t + r * NT;
        const int d = (k1 - klo) & (M - 1);
        const float2 gx = make_float2(acc[r].x * g, acc[r].y * g);
        if (stage_f) stage_f[row + d] = gx;
        if (stage_q) {
            const float qr = fminf(fmaxf(rintf(gx.x), -127.f), 127.f);
            const float qi = fminf(fmaxf(rintf(gx.y), -127.f), 127.f);
            const int16_t packed = (int16_t)(((int)qi << 8) | ((int)qr & 0xff));
            reinterpret_cast<int16_t *>(stage_q)[row + d] = packed;
        }
    }
}

// [n_in][n_spec][C] complex int8 -> [C][n_in][2][n_spec] int8, through a 64 x 64 LDS tile.
__global__ __launch_bounds__(256) void corner_turn_q_kernel(const int16_t *__restrict__ stage, int n_in,
                                                            int n_spec, int n_chan,
                                                            int8_t *__restrict__ out) {
    __shared__ int16_t tile[64][65];
    const int i = blockIdx.y;
    const int n_cb = (n_chan + 63) / 64;
    const int cb = blockIdx.x % n_cb, sb = blockIdx.x / n_cb;
    const int c0 = cb * 64, s0 = sb * 64;
    const int t = threadIdx.x;
    for (int e = t; e < 64 * 64; e += 256) {
        const int sl = e / 64, cl = e % 64;
        const int s = s0 + sl, c = c0 + cl;
        tile[sl][cl] = (s < n_spec && c < n_chan) ? stage[((size_t)i * n_spec + s) * n_chan + c] : 0;
    }
    __syncthreads();
    // write: for each (channel, component), 64 consecutive spectra
    for (int e = t; e < 64 * 2 * 64; e += 256) {
        const int sl = e % 64, comp = (e / 64) % 2, cl = e / 128;
        const int s = s0 + sl, c = c0 + cl;
        if (s < n_spec && c < n_chan) {
            const int16_t v = tile[sl][cl];
            const int8_t b = comp ? (int8_t)(v >> 8) : (int8_t)(v & 0xff);
            out[(((size_t)c * n_in + i) * 2 + comp) * n_spec + s] = b;
        }
    }
}

__global__ __launch_bounds__(256) void corner_turn_f_kernel(const float2 *__restrict__ stage, int n_in,
                                                            int n_spec, int n_chan,
                                                            float *__restrict__ out) {
    __shared__ float2 tile[64][65];
    const int i = blockIdx.y;
    const int n_cb = (n_chan + 63) / 64;
    const int cb = blockIdx.x % n_cb, sb = blockIdx.x / n_cb;
    const int c0 = cb * 64, s0 = sb * 64;
    const int t = threadIdx.x;
    for (int e = t; e < 64 * 64; e += 256) {
        const int sl = e / 64, cl = e % 64;
        const int s = s0 + sl, c = c0 + cl;
        tile[sl][cl] = (s < n_spec && c < n_chan) ? stage[((size_t)i * n_spec + s) * n_chan + c]
                                                  : make_float2(0.f, 0.f);
    }
    __syncthreads();
    for (int e = t; e < 64 * 2 * 64; e += 256) {
        const int sl = e % 64, comp = (e / 64) % 2, cl = e / 128;
        const int s = s0 + sl, c = c0 + cl;
        if (s < n_spec && c < n_chan) {
            const float2 v = tile[sl][cl];
            out[(((size_t)c * n_in + i) * 2 + comp) * n_spec + s] = comp ? v.y : v.x;
        }
    }
}

template <int LOGM>
hipError_t launch_logm(const int8_t *volt, int n_in, int log_n, int n_spec, int klo, int n_chan,
                       const float *gain, int8_t *stage_q, float *stage_f, hipStream_t st) {
    dim3 grid((unsigned)n_in * (unsigned)n_spec);
    hipLaunchKernelGGL(channelize_kernel<LOGM>, grid, dim3((1 << LOGM) / 16), 0, st, volt, log_n,
                       n_spec, klo, n_chan, gain, stage_q, reinterpret_cast<float2 *>(stage_f));
    return hipGetLastError();
}

}  // namespace

// Sub-transform size: the whole transform up to 4096 points, else the smallest power of two
// >= max(4096, n_chan).
int channelize_log_m(int log_n, int n_chan) {
    if (log_n <= 12) return log_n;
    int lm = 12;
    while ((1 << lm) < n_chan) lm++;
    return lm;
}

hipError_t launch_channelize(const int8_t *volt, int n_in, int log_n, int n_spec, int klo,
                             int n_chan, const float *gain, int8_t *stage_q, float *stage_f,
                             hipStream_t st) {
    switch (channelize_log_m(log_n, n_chan)) {
        case 8: return launch_logm<8>(volt, n_in, log_n, n_spec, klo, n_chan, gain, stage_q, stage_f, st);
        case 9: return launch_logm<9>(volt, n_in, log_n, n_spec, klo, n_chan, gain, stage_q, stage_f, st);
        case 10: return launch_logm<10>(volt, n_in, log_n, n_spec, klo, n_chan, gain, stage_q, stage_f, st);
        case 11: return launch_logm<11>(volt, n_in, log_n, n_spec, klo, n_chan, gain, stage_q, stage_f, st);
        case 12: return launch_logm<12>(volt, n_in, log_n, n_spec, klo, n_chan, gain, stage_q, stage_f, st);
        case 13: return launch_logm<13>(volt, n_in, log_n, n_spec, klo, n_chan, gain, stage_q, stage_f, st);
        case 14: return launch_logm<14>(volt, n_in, log_n, n_spec, klo, n_chan, gain, stage_q, stage_f, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_corner_turn_q(const int8_t *stage, int n_in, int n_spec, int n_chan, int8_t *out,
                                hipStream_t st) {
    dim3 grid((unsigned)(((n_chan + 63) / 64) * ((n_spec + 63) / 64)), (unsigned)n_in);
    hipLaunchKernelGGL(corner_turn_q_kernel, grid, dim3(256), 0, st,
                       reinterpret_cast<const int16_t *>(stage), n_in, n_spec, n_chan, out);
    return hipGetLastError();
}

hipError_t launch_corner_turn_f(const float *stage, int n_in, int n_spec, int n_chan, float *out,
                                hipStream_t st) {
    dim3 grid((unsigned)(((n_chan + 63) / 64) * ((n_spec + 63) / 64)), (unsigned)n_in);
    hipLaunchKernelGGL(corner_turn_f_kernel, grid, dim3(256), 0, st,
                       reinterpret_cast<const float2 *>(stage), n_in, n_spec, n_chan, out);
    return hipGetLastError();
}
