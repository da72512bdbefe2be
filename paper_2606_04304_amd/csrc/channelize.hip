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

#include <algorithm>


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

// Build the transform tables of one sub-band in LDS: the two-level table of W_N and the
// [P][16][2] accumulation twiddles W_N^{p (NT r + M j_sel)}.  The kept output of residue
// k1 = t + NT r is k = k1 + M j with j = jl (k1 >= klo mod M) or jl + 1 (k1 < klo mod M), so
// W_N^{p k} = W_N^{p t} * W_N^{p (NT r + M j)}.
template <int LOGM>
__device__ __forceinline__ TwiddleTable chan_tables(float2 *dyn, int log_n, int klo, int t) {
    using PL = Plan<LOGM>;
    constexpr int M = PL::M, NT = PL::NT;
    const int N = 1 << log_n, P = N >> LOGM;
    const int lo_bits = (log_n + 1) >> 1;
    float2 *tw_lo = dyn, *tw_hi = dyn + (1 << lo_bits);
    float2 *acc_tw = tw_hi + (1 << (log_n - lo_bits));
    const TwiddleTable tw = build_twiddles(tw_lo, tw_hi, log_n, t, NT);
    __syncthreads();
    const int jl = klo >> LOGM;
    if (P > 1) {
        for (int e = t; e < P * 32; e += NT) {
            const int p = e >> 5, r = (e >> 1) & 15, sel = e & 1;
            const int j = (jl + sel) & (P - 1);
            acc_tw[e] = tw((p * (NT * r + M * j)) & (N - 1));
        }
    }
    __syncthreads();
    return tw;
}

// size in float2 of the dynamic LDS of one sub-band's tables
__host__ __device__ inline int chan_dyn_elems(int log_n, int log_m) {
    const int lo_bits = (log_n + 1) >> 1;
    const int P = 1 << (log_n - log_m);
    return (1 << lo_bits) + (1 << (log_n - lo_bits)) + (P > 1 ? 32 * P : 0);
}

// One spectrum (input i, spectrum s) of one sub-band: window, P sub-transforms, twiddled
// accumulation of the kept band, gain, float32 and int8 outputs to the staging arrays.
template <int LOGM, int G>
__device__ __forceinline__ void channelize_spectrum(const ChanJob &jb, int i, int s, float2 *buf, const float2 *dyn,
                                                    const TwiddleTable &tw) {
    using PL = Plan<LOGM>;
    constexpr int M = PL::M, NT = PL::NT, R0 = PL::R0;
    constexpr int DW = G >= 4 ? G / 2 : 1;  // dwords of raw samples per element
    static_assert(G == 1 || G == 2 || G == 4 || G == 8, "load grouping");
    const int t = threadIdx.x;
    const int log_n = jb.log_n, n_spec = jb.n_spec, klo = jb.klo, n_chan = jb.n_chan;
    const int N = 1 << log_n;
    const int P = N >> LOGM;
    const int log_p = log_n - LOGM;
    const int lo_bits = (log_n + 1) >> 1;
    const float2 *acc_tw = dyn + (1 << lo_bits) + (1 << (log_n - lo_bits));
    const int rl = klo & (M - 1);
    // raw buffer over this spectrum's samples: one per-thread offset plus scalar offsets per
    // element, with hardware range checking (reads past the spectrum return 0)
    const int16_t *x = reinterpret_cast<const int16_t *>(jb.volt) + ((size_t)i * n_spec + s) * (size_t)N;
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
        // raw samples of G consecutive sub-transforms (one 2G-byte load per element: the G
        // samples x[p0 .. p0 + G - 1 + P m] are adjacent), element m = t + NT b + (M/R0) r.
        // Loading G sub-transforms' samples at once means each 32-byte segment of the spectrum
        // is fetched P/G times rather than P/2 times when the workgroups' spectra overflow L2.
        unsigned raw[E][DW];
#pragma unroll
        for (int b = 0; b < E / R0; b++)
#pragma unroll
            for (int r = 0; r < R0; r++) {
                const int soff = 2 * (p0 + ((NT * b + r * (M / R0)) << log_p));
                unsigned *w = raw[b * R0 + r];
                if constexpr (G == 8) {
                    const auto x = __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff, soff, 0);
                    w[0] = x[0];
                    w[1] = x[1];
                    w[2] = x[2];
                    w[3] = x[3];
                } else if constexpr (G == 4) {
                    const auto x = __builtin_amdgcn_raw_buffer_load_b64(rsrc, voff, soff, 0);
                    w[0] = x[0];
                    w[1] = x[1];
                } else if constexpr (G == 2) {
                    w[0] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, voff, soff, 0);
                } else {
                    w[0] = __builtin_amdgcn_raw_buffer_load_b16(rsrc, voff, soff, 0);
                }
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
                    const int sample = (int)raw[b * R0 + r][0];  // low 16 bits: sub-transform p
                    const float re = (float)(int8_t)(sample & 0xff), im = (float)(int8_t)((sample >> 8) & 0xff);
                    v[b * R0 + r] = make_float2(w * re, w * im);
                }
            // move the next sub-transform's samples into the low 16 bits
            if constexpr (G >= 2) {
#pragma unroll
                for (int e = 0; e < E; e++) {
#pragma unroll
                    for (int w = 0; w + 1 < DW; w++) raw[e][w] = __builtin_amdgcn_alignbit(raw[e][w + 1], raw[e][w], 16);
                    raw[e][DW - 1] >>= 16;
                }
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

    const float g = jb.gain[i];
    const size_t rowo = ((size_t)i * n_spec + s) * (size_t)n_chan;
    unsigned fl = 0;  // NBSI_FLAG_SPEC_* met by this thread
#pragma unroll
    for (int r = 0; r < E; r++) {
        if (!(kept & (1u << r))) continue;
        const int k1 = t + r * NT;
        const int d = (k1 - klo) & (M - 1);
        const float2 gx = make_float2(acc[r].x * g, acc[r].y * g);
        const bool fin = __builtin_isfinite(gx.x) && __builtin_isfinite(gx.y);
        fl |= fin ? 0u : NBSI_FLAG_SPEC_NONFINITE;
        if (jb.stage_f) jb.stage_f[rowo + d] = gx;
        if (jb.stage_q) {
            // a non-finite value has no code: it is requantised to 0 (and flagged)
            const float rr = fin ? rintf(gx.x) : 0.f, ri = fin ? rintf(gx.y) : 0.f;
            fl |= (fabsf(rr) > 127.f || fabsf(ri) > 127.f) ? NBSI_FLAG_SPEC_CLIPPED : 0u;
            const float qr = fminf(fmaxf(rr, -127.f), 127.f);
            const float qi = fminf(fmaxf(ri, -127.f), 127.f);
            const int16_t packed = (int16_t)(((int)qi << 8) | ((int)qr & 0xff));
            reinterpret_cast<int16_t *>(jb.stage_q)[rowo + d] = packed;
        }
    }
    if (fl && jb.flags) atomicOr(jb.flags, fl);
}

template <int LOGM, int G>
__global__ __launch_bounds__((1 << LOGM) / 16) void channelize_kernel(ChanJob jb) {
    __shared__ float2 buf[padded_size(1 << LOGM)];
    extern __shared__ float2 dyn[];  // tables (chan_tables)
    const TwiddleTable tw = chan_tables<LOGM>(dyn, jb.log_n, jb.klo, threadIdx.x);
    channelize_spectrum<LOGM, G>(jb, blockIdx.x / jb.n_spec, blockIdx.x % jb.n_spec, buf, dyn, tw);
}

// Several sub-bands of one transform size in one launch: jobs[j] owns tasks (spectra)
// [task0, task0 + n_in n_spec), one workgroup per task, so the kernel keeps the register
// budget and occupancy of the single-band kernel and the dispatcher balances the workgroups.
template <int LOGM, int G>
__global__ __launch_bounds__((1 << LOGM) / 16) void channelize_batch_kernel(const ChanJob *__restrict__ jobs,
                                                                            int n_jobs, int n_tasks) {
    __shared__ float2 buf[padded_size(1 << LOGM)];
    extern __shared__ float2 dyn[];
    const int task = blockIdx.x;
    if (task >= n_tasks) return;
    int j = 0;
    while (j + 1 < n_jobs && jobs[j + 1].task0 <= task) j++;
    const ChanJob jb = jobs[j];
    const TwiddleTable tw = chan_tables<LOGM>(dyn, jb.log_n, jb.klo, threadIdx.x);
    const int local = task - jb.task0;
    channelize_spectrum<LOGM, G>(jb, local / jb.n_spec, local % jb.n_spec, buf, dyn, tw);
}

// [n_in][n_spec][C] complex int8 -> [C][n_in][2][n_spec] int8, through a 64 x 64 LDS tile:
// tile (i, channel block cb, spectrum block sb).  The tile's rows are read as channel pairs
// (4 bytes) when n_chan is even; each (channel, component) run of spectra is written 16 bytes at
// a time (one vector store when n_spec is a multiple of 16, so the run is 16-byte aligned).
__device__ __forceinline__ void corner_turn_q_tile(const int16_t *__restrict__ stage, int n_in, int n_spec,
                                                   int n_chan, int8_t *__restrict__ out, int i, int cb, int sb,
                                                   int16_t (*tile)[66]) {
    const int c0 = cb * 64, s0 = sb * 64;
    const int S = min(64, n_spec - s0);  // spectra of this tile
    const int t = threadIdx.x;
    const int16_t *src = stage + ((size_t)i * n_spec + s0) * n_chan + c0;
    if ((n_chan & 1) == 0) {
        for (int e = t; e < S * 32; e += 256) {
            const int sl = e >> 5, cp = 2 * (e & 31);
            int v = 0;
            if (c0 + cp < n_chan) v = *reinterpret_cast<const int *>(src + (size_t)sl * n_chan + cp);
            tile[sl][cp] = (int16_t)(v & 0xffff);
            tile[sl][cp + 1] = (int16_t)(v >> 16);
        }
    } else {
        for (int e = t; e < S * 64; e += 256) {
            const int sl = e >> 6, cl = e & 63;
            tile[sl][cl] = c0 + cl < n_chan ? src[(size_t)sl * n_chan + cl] : (int16_t)0;
        }
    }
    __syncthreads();
    // pieces of 16 spectra: piece fastest, then component, then channel (a channel's two runs
    // are adjacent in the output)
    const int NP = (S + 15) >> 4;
    const bool vec = (n_spec & 15) == 0;
    for (int e = t; e < 128 * NP; e += 256) {
        const int piece = e % NP, comp = (e / NP) & 1, cl = e / (2 * NP);
        const int c = c0 + cl;
        if (c >= n_chan) continue;
        const int sl0 = 16 * piece;
        int8_t *dst = out + (((size_t)c * n_in + i) * 2 + comp) * n_spec + s0 + sl0;
        if (vec && sl0 + 16 <= S) {
            int w[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                int x = 0;
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const int v = tile[sl0 + 4 * q + k][cl];
                    x |= ((comp ? (v >> 8) : v) & 0xff) << (8 * k);
                }
                w[q] = x;
            }
            *reinterpret_cast<int4 *>(dst) = make_int4(w[0], w[1], w[2], w[3]);
        } else {
            for (int k = 0; k < 16 && sl0 + k < S; k++) {
                const int16_t v = tile[sl0 + k][cl];
                dst[k] = comp ? (int8_t)(v >> 8) : (int8_t)(v & 0xff);
            }
        }
    }
}

__global__ __launch_bounds__(256) void corner_turn_q_kernel(const int16_t *__restrict__ stage, int n_in,
                                                            int n_spec, int n_chan,
                                                            int8_t *__restrict__ out) {
    __shared__ int16_t tile[64][66];
    const int n_cb = (n_chan + 63) / 64;
    corner_turn_q_tile(stage, n_in, n_spec, n_chan, out, blockIdx.y, blockIdx.x % n_cb, blockIdx.x / n_cb, tile);
}

// Corner turn of several sub-bands: one workgroup per (job, input, 64 x 64 tile) task.
__global__ __launch_bounds__(256) void corner_turn_q_batch_kernel(const ChanJob *__restrict__ jobs, int n_jobs,
                                                                  const int *__restrict__ task0, int n_tasks,
                                                                  int8_t *const *__restrict__ outs, int n_in) {
    __shared__ int16_t tile[64][66];
    const int task = blockIdx.x;
    if (task >= n_tasks) return;
    int j = 0;
    while (j + 1 < n_jobs && task0[j + 1] <= task) j++;
    const ChanJob jb = jobs[j];
    const int local = task - task0[j];
    const int n_cb = (jb.n_chan + 63) / 64, n_sb = (jb.n_spec + 63) / 64;
    const int i = local / (n_cb * n_sb), rem = local % (n_cb * n_sb);
    corner_turn_q_tile(reinterpret_cast<const int16_t *>(jb.stage_q), n_in, jb.n_spec, jb.n_chan, outs[j], i,
                       rem % n_cb, rem / n_cb, tile);
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
hipError_t launch_logm(const ChanJob &jb, int n_in, hipStream_t st) {
    dim3 grid((unsigned)n_in * (unsigned)jb.n_spec);
    const int P = 1 << (jb.log_n - LOGM);
    const size_t lds = sizeof(float2) * chan_dyn_elems(jb.log_n, LOGM);
    if constexpr (LOGM >= 14) {  // 1024 threads leave 128 VGPRs: wider loads would spill
        if (P >= 2)
            hipLaunchKernelGGL((channelize_kernel<LOGM, 2>), grid, dim3((1 << LOGM) / 16), lds, st, jb);
        else
            hipLaunchKernelGGL((channelize_kernel<LOGM, 1>), grid, dim3((1 << LOGM) / 16), lds, st, jb);
    } else if constexpr (LOGM >= 12) {
        if (P >= 8)
            hipLaunchKernelGGL((channelize_kernel<LOGM, 8>), grid, dim3((1 << LOGM) / 16), lds, st, jb);
        else if (P == 4)
            hipLaunchKernelGGL((channelize_kernel<LOGM, 4>), grid, dim3((1 << LOGM) / 16), lds, st, jb);
        else if (P == 2)
            hipLaunchKernelGGL((channelize_kernel<LOGM, 2>), grid, dim3((1 << LOGM) / 16), lds, st, jb);
        else
            hipLaunchKernelGGL((channelize_kernel<LOGM, 1>), grid, dim3((1 << LOGM) / 16), lds, st, jb);
    } else {
        if (P != 1) return hipErrorInvalidValue;  // a transform shorter than 4096 is never split
        hipLaunchKernelGGL((channelize_kernel<LOGM, 1>), grid, dim3((1 << LOGM) / 16), lds, st, jb);
    }
    return hipGetLastError();
}

template <int LOGM, int G>
hipError_t launch_batch_logm(const ChanJob *d_jobs, int n_jobs, int n_tasks, size_t lds,
                             hipStream_t st) {
    hipLaunchKernelGGL((channelize_batch_kernel<LOGM, G>), dim3(n_tasks), dim3((1 << LOGM) / 16), lds, st, d_jobs,
                       n_jobs, n_tasks);
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
                             hipStream_t st, unsigned *flags) {
    ChanJob jb{volt, gain, stage_q, reinterpret_cast<float2 *>(stage_f), log_n, n_spec, klo, n_chan, 0, flags};
    switch (channelize_log_m(log_n, n_chan)) {
        case 8: return launch_logm<8>(jb, n_in, st);
        case 9: return launch_logm<9>(jb, n_in, st);
        case 10: return launch_logm<10>(jb, n_in, st);
        case 11: return launch_logm<11>(jb, n_in, st);
        case 12: return launch_logm<12>(jb, n_in, st);
        case 13: return launch_logm<13>(jb, n_in, st);
        case 14: return launch_logm<14>(jb, n_in, st);
        default: return hipErrorInvalidValue;
    }
}

// Jobs that share one sub-transform size and load grouping (log_m, g) run in one launch
// (one workgroup per spectrum); d_jobs holds them with consecutive task ranges.
hipError_t launch_channelize_batch(const ChanJob *d_jobs, int n_jobs, int n_tasks, int log_m, int g,
                                   int max_dyn_elems, hipStream_t st) {
    const size_t lds = sizeof(float2) * (size_t)max_dyn_elems;
#define NBSI_CB1(LM) \
    case LM: return g == 1 ? launch_batch_logm<LM, 1>(d_jobs, n_jobs, n_tasks, lds, st) : hipErrorInvalidValue;
#define NBSI_CBG(LM)                                                                                  \
    case LM:                                                                                          \
        switch (g) {                                                                                  \
            case 1: return launch_batch_logm<LM, 1>(d_jobs, n_jobs, n_tasks, lds, st); \
            case 2: return launch_batch_logm<LM, 2>(d_jobs, n_jobs, n_tasks, lds, st); \
            case 4: return launch_batch_logm<LM, 4>(d_jobs, n_jobs, n_tasks, lds, st); \
            case 8: return launch_batch_logm<LM, 8>(d_jobs, n_jobs, n_tasks, lds, st); \
            default: return hipErrorInvalidValue;                                                     \
        }
    switch (log_m) {
        NBSI_CB1(8) NBSI_CB1(9) NBSI_CB1(10) NBSI_CB1(11) NBSI_CBG(12) NBSI_CBG(13)
        case 14:
            return g == 2   ? launch_batch_logm<14, 2>(d_jobs, n_jobs, n_tasks, lds, st)
                   : g == 1 ? launch_batch_logm<14, 1>(d_jobs, n_jobs, n_tasks, lds, st)
                            : hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
#undef NBSI_CB1
#undef NBSI_CBG
}

int channelize_dyn_elems(int log_n, int log_m) { return chan_dyn_elems(log_n, log_m); }

// Sub-transforms whose samples one load covers: min(8, P) (min(2, P) for 16384-point sub-transforms).
int channelize_group(int log_n, int log_m) { return std::min(log_m >= 14 ? 2 : 8, 1 << (log_n - log_m)); }

int corner_turn_tasks(int n_in, int n_spec, int n_chan) { return n_in * ((n_chan + 63) / 64) * ((n_spec + 63) / 64); }

hipError_t launch_corner_turn_q_batch(const ChanJob *d_jobs, int n_jobs, const int *d_task0, int n_tasks,
                                      int8_t *const *d_outs, int n_in, hipStream_t st) {
    hipLaunchKernelGGL(corner_turn_q_batch_kernel, dim3(n_tasks), dim3(256), 0, st, d_jobs, n_jobs, d_task0, n_tasks,
                       d_outs, n_in);
    return hipGetLastError();
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
