// Upchannelisation (the paper's Sec. 2.1 FFT over the time samples of each coarse channel),
// periodic Hann window, fftshifted channel selection and int8 requantisation, for gfx950.
//
// Design.  Only a contiguous band of C fine channels is kept out of each N-point spectrum,
// so the transform is evaluated as P = N / M sub-transforms of size M >= C on the
// decimated sequences x[p + P m] (m < M):
//     X[k] = sum_p W_N^{p k} Y_p[k mod M],   Y_p = FFT_M(x)[p + P m]
// Each sub-transform lives in LDS + registers of one workgroup (M/16 threads, 16 complex
// values per thread, radix-16 Stockham passes after a first pass of radix R0), and every
// thread accumulates the band bins it owns in registers; nothing of the N-point spectrum ever
// goes to HBM.  A thread loads the samples of G sub-transforms at a time (one load of 2G
// bytes per element).
//
// The periodic Hann window w[n] = 1/2 - 1/2 cos(2 pi n / N) is the sum of three complex
// exponentials, so windowing the samples equals the three-tap kernel (-1/4, 1/2, -1/4) over
// adjacent bins of the unwindowed spectrum.  The kernel therefore transforms the raw int8
// samples, accumulates the C + 2 bins klo - 1 .. klo + C, and applies the window once per
// spectrum in LDS: no per-sample window arithmetic (the kernel is bound by vector
// instruction issue).  Twiddles are float32 roundings of float64 roots: per-pass tables
// (0.5 ulp) for every pass but the last, a two-level table (~1.5 ulp) and short running
// products for the last pass and the accumulation.
//
// The workgroup of input i, spectrum s writes its kept band to a staging array
// [n_in][n_spec][C] (coalesced); a corner-turn kernel then produces the correlator layout
// [C][n_in][2][n_spec].
#include "internal.h"
#include "fft_dev.h"

#include <algorithm>
#include <type_traits>


namespace {

constexpr int E = 16;  // complex values per thread

template <int LOGM>
struct Plan {
    static constexpr int M = 1 << LOGM;
    static constexpr int NT = M / E;
    static constexpr int R0 = (LOGM % 4 == 0) ? 16 : (1 << (LOGM % 4));  // first radix
    static constexpr int NPASS = (LOGM % 4 == 0) ? LOGM / 4 - 1 : LOGM / 4;  // radix-16 passes
    // transforms of 4096 points or more can be split (P > 1); the last pass then carries the
    // factor W_N^{p t} of the accumulation
    static constexpr bool FOLD = LOGM >= 12;
};

// acc + a * b with two fused multiply-adds per component
__device__ __forceinline__ float2 cmac(float2 acc, float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y)));
}

// Dynamic LDS of one sub-band, in float2 elements: the two-level W_N table (lo at 0, hi), the
// twiddles of the radix-16 passes but the last (tab; pass q, of span 16 ns_q, at
// tab + sum_{q' < q} 16 ns_q'), and for split transforms the accumulation twiddles
// (acc, [P][16][2]), the edge-bin twiddles (ext, [P][2]) and a 2 x 16 exchange slot (eb).
struct ChanLds {
    int hi, tab, acc, ext, eb, total;
};

__host__ __device__ inline ChanLds chan_lds(int log_n, int log_m) {
    constexpr int e = E;
    const int lo_bits = (log_n + 1) >> 1;
    const int r0 = (log_m % 4 == 0) ? 16 : 1 << (log_m % 4);
    const int npass = (log_m % 4 == 0) ? log_m / 4 - 1 : log_m / 4;
    const int P = 1 << (log_n - log_m);
    int ntab = 0;
    for (int q = 0, ns = r0; q + 1 < npass; q++, ns *= e) ntab += e * ns;
    ChanLds l;
    l.hi = 1 << lo_bits;
    l.tab = l.hi + (1 << (log_n - lo_bits));
    l.acc = l.tab + ntab;
    l.ext = l.acc + (P > 1 ? 2 * e * P : 0);
    l.eb = l.ext + (P > 1 ? 2 * P : 0);
    l.total = l.eb + (P > 1 ? 2 * e : 0);
    return l;
}

// A radix-R pass from a table: v[r] *= col[r * ns] (col = table + (t mod ns), entries
// W_{R ns}^{k r} at [r][k]), then the R-point DFT.
template <int R>
__device__ __forceinline__ void pass_tab(float2 *v, const float2 *col, int ns) {
#pragma unroll
    for (int r = 1; r < R; r++) v[r] = cmul(v[r], col[r * ns]);
    dft_r<R>(v);
}

// The last radix-R pass, for one butterfly per thread (j = t): v[r] *= c w^r with
// w = W_{R ns}^{j mod ns}, then the R-point DFT.  Since the DFT is linear, c scales all R
// outputs (FOLD; otherwise c = 1).  w^1..w^7 come by a running product and, for R = 16,
// w^8 = ((w^2)^2)^2, so no chain is longer than about ten roundings.
template <int R, bool FOLD>
__device__ __forceinline__ void pass_run(float2 *v, int t, int ns, int log_n, const TwiddleTable &tw, float2 c) {
    const int k = t & (ns - 1);
    const int sh = log_n - (31 - __clz(ns * R));
    const float2 w = tw(k << sh);
    float2 cur = w;
    if constexpr (FOLD) {
        v[0] = cmul(v[0], c);
        cur = cmul(c, w);
    }
#pragma unroll
    for (int r = 1; r < 8; r++) {
        v[r] = cmul(v[r], cur);
        cur = cmul(cur, w);
    }
    if constexpr (R == 16) {
        const float2 w2 = cmul(w, w), w4 = cmul(w2, w2);
        cur = cmul(w4, w4);
        if constexpr (FOLD) cur = cmul(c, cur);
#pragma unroll
        for (int r = 8; r < 16; r++) {
            v[r] = cmul(v[r], cur);
            cur = cmul(cur, w);
        }
    }
    dft_r<R>(v);
}

// Build the tables of one sub-band in LDS (layout chan_lds).  The unwindowed band starts at
// blo = klo - 1; residue k1 = t + NT r holds band bin k = k1 + M j with j = jl (k1 >= blo
// mod M) or jl + 1 (k1 < blo mod M), so W_N^{p k} = W_N^{p t} * acc[p][r][j - jl], the first
// factor folded into the last pass.  The band's last min(C + 2 - M, 2) bins blo + M + x share
// residue blo + x with the first ones and get their own accumulators; the thread holding that
// residue, t_x = (blo + x) mod NT, carries W_N^{p t_x}, so ext[p][x] = W_N^{p (blo + M + x - t_x)}.
template <int LOGM>
__device__ __forceinline__ TwiddleTable chan_tables(float2 *dyn, int log_n, int klo, int t) {
    using PL = Plan<LOGM>;
    constexpr int M = PL::M, NT = PL::NT;
    const int N = 1 << log_n, P = N >> LOGM;
    const ChanLds L = chan_lds(log_n, LOGM);
    const TwiddleTable tw = build_twiddles(dyn, dyn + L.hi, log_n, t, NT);
    {
        int off = L.tab;
#pragma unroll
        for (int q = 0, ns = PL::R0; q + 1 < PL::NPASS; q++, ns *= E) {
            for (int e = t; e < E * ns; e += NT) {
                const int r = e / ns, k = e % ns;
                double s, c;
                sincospi(-2.0 * (double)(k * r) / (double)(E * ns), &s, &c);
                dyn[off + e] = make_float2((float)c, (float)s);
            }
            off += E * ns;
        }
    }
    __syncthreads();
    if (P > 1) {
        const int blo = (klo - 1) & (N - 1);
        const int jl = blo >> LOGM;
        for (int e = t; e < P * 2 * E; e += NT) {
            const int p = e / (2 * E), r = (e >> 1) % E, sel = e & 1;
            const int j = (jl + sel) & (P - 1);
            dyn[L.acc + e] = tw((p * (NT * r + M * j)) & (N - 1));
        }
        for (int e = t; e < 2 * P; e += NT) {
            const int p = e >> 1, x = e & 1;
            const int tx = (blo + x) & (NT - 1);
            dyn[L.ext + e] = tw((p * (blo + M + x - tx)) & (N - 1));
        }
    }
    __syncthreads();
    return tw;
}

// The raw samples of sub-transform p from half H of word W of each element (H = 0: the low 16
// bits), the first pass and the radix-16 passes; on return v[r] = c Y_p[t + r NT].
template <int LOGM, int H, int W, int DW>
__device__ __forceinline__ void sub_transform(float2 *v, const unsigned (&raw)[E][DW], float2 *buf,
                                              const float2 *tab, const TwiddleTable &tw, int log_n, float2 c) {
    using PL = Plan<LOGM>;
    constexpr int NT = PL::NT, R0 = PL::R0;
    const int t = threadIdx.x;
#pragma unroll
    for (int e = 0; e < E; e++) {
        const unsigned s = raw[e][W] >> (16 * H);
        v[e] = make_float2((float)(int8_t)(s & 0xff), (float)(int8_t)((s >> 8) & 0xff));
    }
    // first pass (radix R0, no twiddles)
#pragma unroll
    for (int b = 0; b < E / R0; b++) dft_r<R0>(v + b * R0);
    __syncthreads();  // buf free (previous sub-transform done reading)
    stockham_store<R0, E>(buf, v, t, NT, 1);
    __syncthreads();
    int ns = R0;
    const float2 *tq = tab;
#pragma unroll
    for (int pass = 0; pass < PL::NPASS; pass++) {
        stockham_load<E, E>(buf, v, t, NT, LOGM);
        if (pass + 1 < PL::NPASS) {
            pass_tab<E>(v, tq + (t & (ns - 1)), ns);
            tq += E * ns;
            __syncthreads();
            stockham_store<E, E>(buf, v, t, NT, ns);
            __syncthreads();
        } else {
            pass_run<E, PL::FOLD>(v, t, ns, log_n, tw, c);
        }
        ns *= E;
    }
}

// One spectrum (input i, spectrum s) of one sub-band: P sub-transforms of the raw samples,
// twiddled accumulation of the band bins klo - 1 .. klo + C, the window as a three-tap kernel
// over them, gain, float32 and int8 outputs to the staging arrays.
template <int LOGM, int G>
__device__ __forceinline__ void channelize_spectrum(const ChanJob &jb, int i, int s, float2 *buf, const float2 *dyn,
                                                    const TwiddleTable &tw) {
    using PL = Plan<LOGM>;
    constexpr int M = PL::M, NT = PL::NT, R0 = PL::R0;
    constexpr int DW = G >= 4 ? G / 2 : 1;  // words of raw samples per element
    static_assert(G == 1 || G == 2 || G == 4 || G == 8, "load grouping");
    const int t = threadIdx.x;
    const int log_n = jb.log_n, n_spec = jb.n_spec, klo = jb.klo, n_chan = jb.n_chan;
    const int N = 1 << log_n;
    const int P = N >> LOGM;
    const int log_p = log_n - LOGM;
    const ChanLds L = chan_lds(log_n, LOGM);
    const float2 *tab = dyn + L.tab;
    const int blo = (klo - 1) & (N - 1);
    const int rl = blo & (M - 1);
    const int n_edge = P > 1 ? min(max(n_chan + 2 - M, 0), 2) : 0;
    const int tx0 = blo & (NT - 1), tx1 = (blo + 1) & (NT - 1);
    const int rx0 = rl / NT, rx1 = ((blo + 1) & (M - 1)) / NT;
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
    float2 xa0 = make_float2(0.f, 0.f), xa1 = make_float2(0.f, 0.f);  // edge bins (lanes tx0, tx1)

    // accumulate sub-transform p (v = W_N^{p t} Y_p[t + r NT] when split)
    auto accumulate = [&](const float2 *v, int p) {
        if (P == 1) {
#pragma unroll
            for (int r = 0; r < E; r++) acc[r] = v[r];
            return;
        }
        const float2 *row = dyn + L.acc + p * 2 * E;
#pragma unroll
        for (int r = 0; r < E; r++) acc[r] = cmac(acc[r], v[r], row[2 * r + ((sel >> r) & 1)]);
        if (n_edge > 0) {
            // the edge residue's register is chosen by a uniform index: its lane passes all E
            // values through LDS and reads the one it needs back
            float2 *eb = const_cast<float2 *>(dyn) + L.eb;
            if (t == tx0) {
#pragma unroll
                for (int r = 0; r < E; r++) eb[r] = v[r];
                xa0 = cmac(xa0, eb[rx0], dyn[L.ext + 2 * p]);
            }
            if (n_edge > 1 && t == tx1) {
#pragma unroll
                for (int r = 0; r < E; r++) eb[E + r] = v[r];
                xa1 = cmac(xa1, eb[E + rx1], dyn[L.ext + 2 * p + 1]);
            }
        }
    };
    // sub-transforms p (low half of word W) and p + 1 (high half)
    auto pair = [&](auto wc, const unsigned (&raw)[E][DW], int p) {
        constexpr int W = decltype(wc)::value;
        float2 v[E];
        const float2 one = make_float2(1.f, 0.f);
        sub_transform<LOGM, 0, W, DW>(v, raw, buf, tab, tw, log_n,
                                         PL::FOLD && P > 1 ? tw((p * t) & (N - 1)) : one);
        accumulate(v, p);
        if constexpr (G >= 2) {
            sub_transform<LOGM, 1, W, DW>(v, raw, buf, tab, tw, log_n,
                                             PL::FOLD && P > 1 ? tw(((p + 1) * t) & (N - 1)) : one);
            accumulate(v, p + 1);
        }
    };

    for (int p0 = 0; p0 < P; p0 += G) {
        // raw samples of G consecutive sub-transforms (2G bytes per element: the G samples
        // x[p0 .. p0 + G - 1 + P m] are adjacent), element m = t + NT b + (M/R0) r.  Loading
        // the samples of G sub-transforms at once means each 32-byte segment of the spectrum is
        // fetched P/G times rather than P/2 times when the workgroups' spectra overflow L2.
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
        // two sub-transforms per step from word 0, then the next word moves down
#pragma unroll 1
        for (int g = 0; g < G; g += 2) {
            pair(std::integral_constant<int, 0>{}, raw, p0 + g);
#pragma unroll
            for (int e = 0; e < E; e++)
#pragma unroll
                for (int w = 0; w + 1 < DW; w++) raw[e][w] = raw[e][w + 1];
        }
    }

    // unwindowed band in LDS: band[q] = X[blo + q] for q < C + 2 (positions M, M + 1 are the
    // edge bins; with P = 1 the spectrum is M-periodic and they wrap to 0, 1)
    __syncthreads();  // every wave is done with buf
#pragma unroll
    for (int r = 0; r < E; r++) {
        const int q = (t + r * NT - blo) & (M - 1);
        if (q < n_chan + 2) buf[q] = acc[r];
    }
    if (n_edge > 0 && t == tx0) buf[M] = xa0;
    if (n_edge > 1 && t == tx1) buf[M + 1] = xa1;
    __syncthreads();

    const float g = jb.gain[i];
    const size_t rowo = ((size_t)i * n_spec + s) * (size_t)n_chan;
    unsigned fl = 0;  // NBSI_FLAG_SPEC_* met by this thread
#pragma unroll
    for (int r = 0; r < E; r++) {
        if (!(kept & (1u << r))) continue;
        const int k1 = t + r * NT;
        const int d = (k1 - klo) & (M - 1);  // output channel; bins d, d + 1, d + 2 of the band
        int qp = d + 2;
        if (P == 1 && qp >= M) qp -= M;
        const float2 xm = buf[d], x0 = buf[d + 1 == M && P == 1 ? 0 : d + 1], xp = buf[qp];
        // window: X_w[k] = X[k] / 2 - (X[k - 1] + X[k + 1]) / 4
        const float2 xw = make_float2(fmaf(-0.25f, xm.x + xp.x, 0.5f * x0.x), fmaf(-0.25f, xm.y + xp.y, 0.5f * x0.y));
        const float2 gx = make_float2(xw.x * g, xw.y * g);
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

// threads per workgroup, and the waves per SIMD the register budget is built for: three
// 256-thread workgroups per CU for 4096-point sub-transforms loaded four at a time (168 VGPRs;
// at 16 sub-transforms per spectrum 8% faster than two workgroups loading eight at a time),
// else the compiler's choice
template <int LOGM, int G>
constexpr int chan_threads() { return (1 << LOGM) / E; }
template <int LOGM, int G>
constexpr int chan_waves() { return LOGM == 12 && G <= 4 ? 3 : 1; }

template <int LOGM, int G>
__global__ __launch_bounds__((chan_threads<LOGM, G>()), (chan_waves<LOGM, G>())) void channelize_kernel(ChanJob jb) {
    __shared__ float2 buf[padded_size(1 << LOGM)];
    extern __shared__ float2 dyn[];  // tables (chan_tables)
    const TwiddleTable tw = chan_tables<LOGM>(dyn, jb.log_n, jb.klo, threadIdx.x);
    channelize_spectrum<LOGM, G>(jb, blockIdx.x / jb.n_spec, blockIdx.x % jb.n_spec, buf, dyn, tw);
}

// Several sub-bands of one transform size in one launch: jobs[j] owns tasks (spectra)
// [task0, task0 + n_in n_spec), one workgroup per task, so the kernel keeps the register
// budget and occupancy of the single-band kernel and the dispatcher balances the workgroups.
template <int LOGM, int G>
__global__ __launch_bounds__((chan_threads<LOGM, G>()), (chan_waves<LOGM, G>())) void channelize_batch_kernel(
    const ChanJob *__restrict__ jobs, int n_jobs, int n_tasks) {
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

// Sub-transforms whose samples one load covers (never more than P).  Each element's 2P bytes
// of samples are fetched P/G times (a spectrum's lines leave L2 between its load groups), so G
// trades fetches against registers: for 4096-point sub-transforms G = 4 (the 168-VGPR budget of
// three workgroups per CU) while P <= 16, and G = 8 (two workgroups) beyond, where the fetches
// of G = 4 bound the kernel (measured at P = 32 / 64: 3.28 / 6.96 ms against 2.48 / 3.34 ms);
// 2 for 16384-point sub-transforms (1024 threads leave 128 VGPRs: wider loads would spill);
// else 8.
int chan_group(int log_n, int log_m) {
    const int P = 1 << (log_n - log_m);
    if (log_m == 12) return std::min(P <= 16 ? 4 : 8, P);
    return std::min(log_m >= 14 ? 2 : 8, P);
}

template <int LOGM, int G>
hipError_t launch_g(const ChanJob &jb, int n_in, hipStream_t st) {
    const size_t lds = sizeof(float2) * chan_lds(jb.log_n, LOGM).total;
    hipLaunchKernelGGL((channelize_kernel<LOGM, G>), dim3((unsigned)n_in * (unsigned)jb.n_spec),
                       dim3(chan_threads<LOGM, G>()), lds, st, jb);
    return hipGetLastError();
}

template <int LOGM>
hipError_t launch_logm(const ChanJob &jb, int n_in, hipStream_t st) {
    if constexpr (LOGM < 12) {
        if (jb.log_n != LOGM) return hipErrorInvalidValue;  // a transform shorter than 4096 is never split
        return launch_g<LOGM, 1>(jb, n_in, st);
    } else {
        switch (chan_group(jb.log_n, LOGM)) {
            case 1: return launch_g<LOGM, 1>(jb, n_in, st);
            case 2: return launch_g<LOGM, 2>(jb, n_in, st);
            case 4:
                if constexpr (LOGM < 14) return launch_g<LOGM, 4>(jb, n_in, st);
                return hipErrorInvalidValue;
            case 8:
                if constexpr (LOGM < 14) return launch_g<LOGM, 8>(jb, n_in, st);
                return hipErrorInvalidValue;
            default: return hipErrorInvalidValue;
        }
    }
}

template <int LOGM, int G>
hipError_t launch_batch_logm(const ChanJob *d_jobs, int n_jobs, int n_tasks, size_t lds,
                             hipStream_t st) {
    hipLaunchKernelGGL((channelize_batch_kernel<LOGM, G>), dim3(n_tasks), dim3(chan_threads<LOGM, G>()), lds, st,
                       d_jobs, n_jobs, n_tasks);
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

int channelize_dyn_elems(int log_n, int log_m) { return chan_lds(log_n, log_m).total; }

int channelize_group(int log_n, int log_m) { return chan_group(log_n, log_m); }

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
