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

// W_16^e = exp(-2 pi i e / 16)
__device__ __forceinline__ float2 w16(int e) {
    constexpr float c[16] = {1.f, 0.92387953251128675613f, 0.70710678118654752440f, 0.38268343236508977173f,
                             0.f, -0.38268343236508977173f, -0.70710678118654752440f, -0.92387953251128675613f,
                             -1.f, -0.92387953251128675613f, -0.70710678118654752440f, -0.38268343236508977173f,
                             0.f, 0.38268343236508977173f, 0.70710678118654752440f, 0.92387953251128675613f};
    return make_float2(c[e & 15], -c[(e + 12) & 15]);  // sin(2 pi e/16) = cos(2 pi (e - 4)/16)
}

// One radix-16 Stockham pass for one butterfly per thread (j = t).  The twiddles w^r,
// w = W_{16 ns}^{j mod ns}, come from one table entry: w^1..w^7 by a running product and
// w^8..w^15 from w^8 = ((w^2)^2)^2, so no chain is longer than about ten roundings.
__device__ __forceinline__ void pass16(float2 *v, int t, int ns, int log_n, const TwiddleTable &tw) {
    if (ns > 1) {
        const int k = t & (ns - 1);
        const int sh = log_n - (31 - __clz(ns * 16));
        const float2 w = tw(k << sh);
        float2 cur = w;
#pragma unroll
        for (int r = 1; r < 8; r++) {
            v[r] = cmul(v[r], cur);
            cur = cmul(cur, w);
        }
        const float2 w2 = cmul(w, w), w4 = cmul(w2, w2);
        cur = cmul(w4, w4);
#pragma unroll
        for (int r = 8; r < 16; r++) {
            v[r] = cmul(v[r], cur);
            cur = cmul(cur, w);
        }
    }
    dft16(v);
}

template <int LOGM, int G>
__global__ __launch_bounds__((1 << LOGM) / 16) void channelize_kernel(
    const int8_t *__restrict__ volt, int log_n, int n_spec, int klo, int n_chan,
    const float *__restrict__ gain, int8_t *__restrict__ stage_q, float2 *__restrict__ stage_f) {
    using PL = Plan<LOGM>;
    constexpr int M = PL::M, NT = PL::NT, R0 = PL::R0;
    __shared__ float2 buf[padded_size(M)];
    // dynamic LDS: two-level table of W_N (2^lo_bits + 2^(log_n - lo_bits) entries), then
    // [P][16][2] accumulation twiddles W_N^{p (NT r + M j_sel)}
    extern __shared__ float2 dyn[];

    const int t = threadIdx.x;
    const int s = blockIdx.x % n_spec;
    const int i = blockIdx.x / n_spec;
    const int N = 1 << log_n;
    const int P = N >> LOGM;
    const int log_p = log_n - LOGM;

    const int lo_bits = (log_n + 1) >> 1;
    float2 *tw_lo = dyn, *tw_hi = dyn + (1 << lo_bits);
    float2 *acc_tw = tw_hi + (1 << (log_n - lo_bits));
    const TwiddleTable tw = build_twiddles(tw_lo, tw_hi, log_n, t, NT);
    __syncthreads();
    // Kept output of residue k1 = t + NT r is k = k1 + M j with j = jl (k1 >= klo mod M) or
    // jl + 1 (k1 < klo mod M), so W_N^{p k} = W_N^{p t} * W_N^{p (NT r + M j)}.
    const int rl = klo & (M - 1), jl = klo >> LOGM;
    if (P > 1) {
        for (int e = t; e < P * 32; e += NT) {
            const int p = e >> 5, r = (e >> 1) & 15, sel = e & 1;
            const int j = (jl + sel) & (P - 1);
            acc_tw[e] = tw((p * (NT * r + M * j)) & (N - 1));
        }
    }
    __syncthreads();

    // raw buffer over this spectrum's samples: one per-thread offset plus scalar offsets per
    // element, with hardware range checking (reads past the spectrum return 0)
    const int16_t *x = reinterpret_cast<const int16_t *>(volt) + ((size_t)i * n_spec + s) * (size_t)N;
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<int16_t *>(x), (short)0, N * 2, 0x00020000);
    const int voff = (t << log_p) * 2;

    unsigned kept = 0, sel = 0;
#pragma unroll
    for (int r = 0; r < E; r++) {
        const int k1 = t + r * NT;
        if (((k1 - klo) & (M - 1)) < n_chan) kept |= 1u << r;
        if (k1 < rl) sel |= 1u << r;
    }

    float2 acc[E];
#pragma unroll
    for (int r = 0; r < E; r++) acc[r] = make_float2(0.f, 0.f);

    for (int p0 = 0; p0 < P; p0 += G) {
        // raw samples of G consecutive sub-transforms: element m = t + NT b + (M/R0) r
        int raw[E];
#pragma unroll
        for (int b = 0; b < E / R0; b++)
#pragma unroll
            for (int r = 0; r < R0; r++) {
                const int soff = 2 * (p0 + ((NT * b + r * (M / R0)) << log_p));
                if constexpr (G == 2) raw[b * R0 + r] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, voff, soff, 0);
                else raw[b * R0 + r] = (int)(int16_t)__builtin_amdgcn_raw_buffer_load_b16(rsrc, voff, soff, 0);
            }
#pragma unroll 1
        for (int g = 0; g < G; g++) {
            const int p = p0 + g;
            float2 v[E];
            // window w[n] = 1/2 - 1/2 cos(2 pi n / N), n = p + P t + (N/16) b + (N/R0) r:
            // cos from W_N^{p + P t} times the constant W_16^{b + (16/R0) r}
            const float2 wb = tw(p + (t << log_p));
#pragma unroll
            for (int b = 0; b < E / R0; b++)
#pragma unroll
                for (int r = 0; r < R0; r++) {
                    const float2 wc = w16(b + (16 / R0) * r);
                    const float cs = wb.x * wc.x - wb.y * wc.y;
                    const float w = 0.5f - 0.5f * cs;
                    const int sample = (G == 2) ? (raw[b * R0 + r] >> (16 * g)) : raw[b * R0 + r];
                    const float re = (float)(int8_t)(sample & 0xff), im = (float)(int8_t)((sample >> 8) & 0xff);
                    v[b * R0 + r] = make_float2(w * re, w * im);
                }
            // first pass (radix R0, no twiddles)
#pragma unroll
            for (int b = 0; b < E / R0; b++) dft_r<R0>(v + b * R0);
            __syncthreads();  // buf free (previous sub-transform done reading)
            stockham_store<R0, E>(buf, v, t, NT, 1);
            __syncthreads();
            int ns = R0;
#pragma unroll
            for (int pass = 0; pass < PL::NPASS16; pass++) {
                stockham_load<16, E>(buf, v, t, NT, LOGM);
                pass16(v, t, ns, log_n, tw);
                if (pass + 1 < PL::NPASS16) {
                    __syncthreads();
                    stockham_store<16, E>(buf, v, t, NT, ns);
                    __syncthreads();
                }
                ns *= 16;
            }
            // v[r] = Y_p[t + r NT]
            if (P == 1) {
#pragma unroll
                for (int r = 0; r < E; r++) acc[r] = v[r];
            } else {
                const float2 bp = tw((p * t) & (N - 1));
                const float2 *row = acc_tw + p * 32;
                // every register accumulates (branch-free); only kept outputs are stored
#pragma unroll
                for (int r = 0; r < E; r++) {
                    const float2 tr = cmul(bp, row[2 * r + ((sel >> r) & 1)]);
                    acc[r] = cadd(acc[r], cmul(v[r], tr));
                }
            }
        }
    }

    const float g = gain[i];
    const size_t rowo = ((size_t)i * n_spec + s) * (size_t)n_chan;
#pragma unroll
    for (int r = 0; r < E; r++) {
        if (!(kept & (1u << r))) continue;
        const int k1 = t + r * NT;
        const int d = (k1 - klo) & (M - 1);
        const float2 gx = make_float2(acc[r].x * g, acc[r].y * g);
        if (stage_f) stage_f[rowo + d] = gx;
        if (stage_q) {
            const float qr = fminf(fmaxf(rintf(gx.x), -127.f), 127.f);
            const float qi = fminf(fmaxf(rintf(gx.y), -127.f), 127.f);
            const int16_t packed = (int16_t)(((int)qi << 8) | ((int)qr & 0xff));
            reinterpret_cast<int16_t *>(stage_q)[rowo + d] = packed;
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
    const int P = 1 << (log_n - LOGM);
    float2 *sf = reinterpret_cast<float2 *>(stage_f);
    const int lo_bits = (log_n + 1) >> 1;
    const size_t lds = sizeof(float2) * ((1 << lo_bits) + (1 << (log_n - lo_bits)) + (P > 1 ? 32 * P : 0));
    if (P >= 2)
        hipLaunchKernelGGL((channelize_kernel<LOGM, 2>), grid, dim3((1 << LOGM) / 16), lds, st, volt, log_n, n_spec,
                           klo, n_chan, gain, stage_q, sf);
    else
        hipLaunchKernelGGL((channelize_kernel<LOGM, 1>), grid, dim3((1 << LOGM) / 16), lds, st, volt, log_n, n_spec,
                           klo, n_chan, gain, stage_q, sf);
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
