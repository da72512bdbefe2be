// All-sky imaging of every fine channel (the paper's Sec. 2.2), gfx950.
//
// I(l, m) = (1/|B|) sum_{b in B} Re[V_I,b exp(-2 pi i (u_b l + v_b m))],  V_I = (V_XX + V_YY)/2.
// Baseline coordinates and the membership test of B are float64 and written with explicit
// rounding intrinsics (no contraction), so the set B is decided identically everywhere.
//
// DFT method: one workgroup per (channel, image row); baselines are staged in LDS in chunks,
// phases are float64 turns reduced to [0, 1) before a float32 sincospi.
//
// GRID method (NUFFT type 1 with the exponential-of-semicircle kernel, width 8, beta = 18.4,
// on a 2x oversampled M = 2 n_pix grid, cell du = 1/4 wavelength):
//   pass A, one workgroup per (channel, band of grid rows): grid the band's baselines into LDS
//     (float32 accumulation; FP32, FP16 or BF16 products), FFT every row along u, keep the
//     n_pix central outputs (image columns) and write them column-major to an intermediate;
//   pass B, one workgroup per (channel, band of image columns): FFT along v, keep the n_pix
//     central outputs (image rows), divide by the kernel's Fourier transform in l and m, scale
//     by 1/|B| and write the real part.
// The grid never leaves LDS; the only HBM round trip is the n_pix x M intermediate.
#include "internal.h"
#include "fft_dev.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

namespace {

constexpr double C_LIGHT = 299792458.0;

struct UV {
    double u, v;
};

__device__ __forceinline__ UV baseline_uv(const double *__restrict__ xyz, int a, int b, double nu) {
    const double dx = __dsub_rn(xyz[3 * a], xyz[3 * b]);
    const double dy = __dsub_rn(xyz[3 * a + 1], xyz[3 * b + 1]);
    UV r;
    r.u = __ddiv_rn(__dmul_rn(dx, nu), C_LIGHT);
    r.v = __ddiv_rn(__dmul_rn(dy, nu), C_LIGHT);
    return r;
}

// Membership of the imaged set B (see nbsi_image_plan_create).
__device__ __forceinline__ bool in_set(UV w, int grid_n_pix, double uv_min, double uv_max) {
    const double r = __dsqrt_rn(__dadd_rn(__dmul_rn(w.u, w.u), __dmul_rn(w.v, w.v)));
    if (r < uv_min || r > uv_max) return false;
    if (grid_n_pix > 0) {
        const double U = (double)(grid_n_pix - 5) * 0.25;
        if (fabs(w.u) > U || fabs(w.v) > U) return false;
    }
    return true;
}

// The gridder's view of the membership bitmap of B (rows of the plan's bitmap from the chunk's
// first channel on).
struct SetTest {
    const unsigned *bits;
    int words;
    __device__ __forceinline__ bool operator()(int c, int k) const {
        return (bits[(size_t)c * words + (k >> 5)] >> (k & 31)) & 1u;
    }
};

// Stokes I of pair (a, b), a > b: (V[t(2a, 2b)] + V[t(2a+1, 2b+1)]) / 2.
template <typename VT>
__device__ __forceinline__ float2 stokes_i(const VT *__restrict__ vc, int a, int b);

template <>
__device__ __forceinline__ float2 stokes_i<int2>(const int2 *__restrict__ vc, int a, int b) {
    const size_t txx = (size_t)(2 * a) * (2 * a + 1) / 2 + 2 * b;
    const size_t tyy = (size_t)(2 * a + 1) * (2 * a + 2) / 2 + 2 * b + 1;
    const int2 x = vc[txx], y = vc[tyy];
    return make_float2((float)(0.5 * ((double)x.x + (double)y.x)), (float)(0.5 * ((double)x.y + (double)y.y)));
}

template <>
__device__ __forceinline__ float2 stokes_i<float2>(const float2 *__restrict__ vc, int a, int b) {
    const size_t txx = (size_t)(2 * a) * (2 * a + 1) / 2 + 2 * b;
    const size_t tyy = (size_t)(2 * a + 1) * (2 * a + 2) / 2 + 2 * b + 1;
    const float2 x = vc[txx], y = vc[tyy];
    return make_float2(0.5f * (x.x + y.x), 0.5f * (x.y + y.y));
}

// ---- |B| per channel, and (gridding plans) the membership bitmap of B ----
// inb[c][k / 32] bit k % 32 = pair k is in B at channel c; words = (n_pairs + 31) / 32.
__global__ __launch_bounds__(256) void count_kernel(const double *__restrict__ xyz, const double *__restrict__ freq,
                                                    const int2 *__restrict__ pairs, int n_pairs, int grid_n_pix,
                                                    double uv_min, double uv_max, int *__restrict__ nb,
                                                    unsigned *__restrict__ inb) {
    __shared__ int part[256];
    const int c = blockIdx.x;
    const double nu = freq[c];
    const int lane = threadIdx.x & 63, words = (n_pairs + 31) >> 5;
    int cnt = 0;
    for (int k0 = 0; k0 < n_pairs; k0 += 256) {  // every lane takes part in the ballot
        const int k = k0 + (int)threadIdx.x;
        bool ok = false;
        if (k < n_pairs) {
            const int2 p = pairs[k];
            ok = in_set(baseline_uv(xyz, p.x, p.y, nu), grid_n_pix, uv_min, uv_max);
        }
        cnt += ok ? 1 : 0;
        if (inb) {
            const unsigned long long m = __ballot(ok);
            const int w = (k - lane) >> 5;  // this wave's first word (k - lane is a multiple of 64)
            if (lane == 0 && w < words) inb[(size_t)c * words + w] = (unsigned)m;
            if (lane == 32 && w + 1 < words) inb[(size_t)c * words + w + 1] = (unsigned)(m >> 32);
        }
    }
    part[threadIdx.x] = cnt;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) nb[c] = part[0];
}

// One atomic per wave that met a non-finite output value.
__device__ __forceinline__ void flag_nonfinite(bool bad, unsigned *flags) {
    if (__ballot(bad) && flags && (threadIdx.x & 63) == 0) atomicOr(flags, NBSI_FLAG_IMAGE_NONFINITE);
}

// ---- direct Fourier imager ----
template <typename VT>
__global__ __launch_bounds__(256) void dft_kernel(const VT *__restrict__ vis, const double *__restrict__ xyz,
                                                  const double *__restrict__ freq, const int2 *__restrict__ pairs,
                                                  int n_pairs, int n_ant, int n_pix, double uv_min, double uv_max,
                                                  const int *__restrict__ nb, float *__restrict__ img,
                                                  unsigned *__restrict__ flags) {
    __shared__ double su[256], sv[256];
    __shared__ float2 sval[256];
    __shared__ int sok[256];
    const int c = blockIdx.y;
    const int y = blockIdx.x;
    const int t = threadIdx.x;
    const double nu = freq[c];
    const size_t nprod = (size_t)(2 * n_ant) * (2 * n_ant + 1) / 2;
    const VT *vc = vis + (size_t)c * nprod;
    const double m = (double)(y - n_pix / 2) * (2.0 / (double)n_pix);
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < n_pairs; k0 += 256) {
        __syncthreads();
        const int k = k0 + t;
        int ok = 0;
        if (k < n_pairs) {
            const int2 p = pairs[k];
            const UV w = baseline_uv(xyz, p.x, p.y, nu);
            ok = in_set(w, 0, uv_min, uv_max);
            su[t] = w.u;
            sv[t] = w.v;
            sval[t] = ok ? stokes_i<VT>(vc, p.x, p.y) : make_float2(0.f, 0.f);
        }
        sok[t] = ok;
        __syncthreads();
        const int kn = min(256, n_pairs - k0);
        for (int q = 0; q < kn; q++) {
            if (!sok[q]) continue;
            const double uq = su[q], vq = sv[q];
            const float2 val = sval[q];
#pragma unroll
            for (int xi = 0; xi < 4; xi++) {
                const int x = t + 256 * xi;
                if (x < n_pix) {
                    const double l = (double)(x - n_pix / 2) * (2.0 / (double)n_pix);
                    const double turns = uq * l + vq * m;
                    const double frac = turns - floor(turns);
                    float sn, cs;
                    sincospif(2.0f * (float)frac, &sn, &cs);
                    acc[xi] += val.x * cs + val.y * sn;
                }
            }
        }
    }
    const int n = nb[c];
    const float inv = n > 0 ? (float)(1.0 / (double)n) : 0.f;
    bool bad = false;
#pragma unroll
    for (int xi = 0; xi < 4; xi++) {
        const int x = t + 256 * xi;
        if (x < n_pix) {
            const float o = acc[xi] * inv;
            bad |= !__builtin_isfinite(o);
            img[((size_t)c * n_pix + y) * n_pix + x] = o;
        }
    }
    flag_nonfinite(bad, flags);
}

// ---- gridding ----
// Gridding tile: a workgroup of 256 threads holds GE complex cells per thread, i.e. a band of
// 256 GE / M grid rows (GE = 16: 32 KB of LDS, four workgroups per CU; GE = 32: 64 KB, two).
// The plan fixes GE (the autotuner chooses it per image size).
template <int GE>
struct Tile {
    static constexpr int CELLS = 256 * GE;
};
constexpr float ES_BETA = 2.30f * 8.0f;

__device__ __forceinline__ float es_kernel(float z) {
    // exp(beta (sqrt(1 - z^2) - 1)) for |z| <= 1, else 0
    const float q = 1.f - z * z;
    return q > 0.f ? expf(ES_BETA * (sqrtf(q) - 1.f)) : 0.f;
}

// The same kernel with the hardware exp2 and square root instructions (about 2 ulp; the
// argument of exp2 is <= 0 and the result is only used in [2^-27, 1], so neither needs the
// library's denormal range handling).
__device__ __forceinline__ float es_kernel_fast(float z) {
    const float q = 1.f - z * z;
    return q > 0.f ? __builtin_amdgcn_exp2f(ES_BETA * 1.44269504088896341f * (__builtin_amdgcn_sqrtf(q) - 1.f)) : 0.f;
}

template <int PREC>
__device__ __forceinline__ float2 grid_product(float2 val, float wu, float wv) {
    if constexpr (PREC == NBSI_PREC_FP16) {
        const __half2 v2 = __floats2half2_rn(val.x, val.y);
        const __half w = __float2half_rn(wu * 1.0f);
        const __half w2 = __float2half_rn(wv);
        const __half ww = __hmul(w, w2);
        const __half2 r = __hmul2(v2, __halves2half2(ww, ww));
        return __half22float2(r);
    } else if constexpr (PREC == NBSI_PREC_BF16) {
        const __hip_bfloat16 vr = __float2bfloat16(val.x), vi = __float2bfloat16(val.y);
        const __hip_bfloat16 ww = __hmul(__float2bfloat16(wu), __float2bfloat16(wv));
        return make_float2(__bfloat162float(__hmul(vr, ww)), __bfloat162float(__hmul(vi, ww)));
    } else {
        const float ww = wu * wv;
        return make_float2(val.x * ww, val.y * ww);
    }
}

// LDS layout of the imager's transform buffers: rows of L complex values, one pad slot after
// every 8 values and 2 more per row.  With it the Stockham passes' loads (consecutive lanes,
// consecutive values) and strided stores (strides of 1, 2, 4, 8 and 64 values x the radix) fall
// in distinct banks, and values of one column in consecutive rows do not share a bank.
// LDS layout of rows of L complex values (L >= 64): element i of row r sits at
//   r RS + (i & ~31) + ((i & 31) ^ (((i >> 5) C1 ^ r C2) & 31)),
// an XOR swizzle of the 32 values (64 banks) of each aligned run.  A run read or written
// contiguously stays conflict-free; the strided accesses of the Stockham passes, the gridding
// accumulators' store, the kept-column read-out and the column pass's tile store and Hermitian
// fold are spread over the banks by the run index and the row.  The constants were chosen per L
// with a bank model of every access pattern of both passes (the eight-byte accesses of a wave in
// two halves of 32 lanes over 64 four-byte banks): about 1.1x the conflict-free cycles, where a
// padding of one value per eight had 1.7-2x.
template <int L>
struct RowLayout {
    static constexpr int C1 = (L == 256 || L >= 1024) ? 9 : 5;
    static constexpr int C2 = L == 128 ? 25 : (L == 2048 ? 0 : 1);
    static constexpr int RS = L + (L == 128 ? 0 : ((L == 512 || L == 1024) ? 4 : 8));
    static_assert(L >= 64, "swizzle runs of 32");
};

template <int L>
__device__ __forceinline__ int lds_at(int row, int i) {
    using RL = RowLayout<L>;
    return row * RL::RS + ((i & ~31) | ((i & 31) ^ ((((i >> 5) * RL::C1) ^ (row * RL::C2)) & 31)));
}

// Radix of pass p of a 2^LOGL-point transform: 8 throughout, after one radix-2 or radix-4 pass
// when LOGL is not a multiple of 3.
template <int LOGL>
struct FftPasses {
    static constexpr int REM = LOGL % 3;
    static constexpr int N = LOGL / 3 + (REM ? 1 : 0);
    static constexpr int log_radix(int p) { return (REM && p == 0) ? REM : 3; }
    static constexpr int log_ns(int p) { return p == 0 ? 0 : (REM ? REM + 3 * (p - 1) : 3 * p); }
};

// W_T^m from the half table tab[m] = W_T^m, m < T / 2 (W_T^(m + T/2) = -W_T^m).
template <int LOGT>
__device__ __forceinline__ float2 twid(const float2 *tab, int m) {
    constexpr int H = 1 << (LOGT - 1);
    const float2 w = tab[m & (H - 1)];
    return (m & H) ? make_float2(-w.x, -w.y) : w;
}

// One Stockham pass (radix 2^LOGR, 2^LOGNS points already combined) over NROWS rows of
// L = 2^LOGL values in LDS, 256 threads, E = NROWS L / 256 values per thread.  Twiddles
// W_{NS R}^{k r} come from the half table of W_T^m (T = 2^LOGT >= L).  Every twiddled pass has
// L / R <= 256 butterflies per row, so all of a thread's butterflies sit at the same position k
// of their rows and share one set of twiddles.
template <int LOGL, int NROWS, int LOGR, int LOGNS, int LOGT>
__device__ __forceinline__ void fft_pass(float2 *buf, const float2 *tab, int t) {
    constexpr int L = 1 << LOGL, R = 1 << LOGR, NS = 1 << LOGNS;
    constexpr int E = NROWS * L / 256, NB = E / R, PER_ROW = L / R;
    static_assert(E % R == 0, "whole butterflies per thread");
    static_assert(NS == 1 || 256 % PER_ROW == 0, "shared twiddles");
    float2 v[E];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int g = t + 256 * b, row = g / PER_ROW, j = g % PER_ROW;
#pragma unroll
        for (int r = 0; r < R; r++) v[b * R + r] = buf[lds_at<L>(row, j + r * PER_ROW)];
    }
    __syncthreads();
    float2 w[R];
    if constexpr (NS > 1) {
        const int k = (t % PER_ROW) & (NS - 1);
#pragma unroll
        for (int r = 1; r < R; r++) w[r] = twid<LOGT>(tab, (k * r) << (LOGT - LOGNS - LOGR));
    }
#pragma unroll
    for (int b = 0; b < NB; b++) {
        if constexpr (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; r++) v[b * R + r] = cmul(v[b * R + r], w[r]);
        }
        dft_r<R>(v + b * R);
        const int g = t + 256 * b, row = g / PER_ROW, j = g % PER_ROW;
        const int base = ((j >> LOGNS) << (LOGNS + LOGR)) + (j & (NS - 1));
#pragma unroll
        for (int r = 0; r < R; r++) buf[lds_at<L>(row, base + r * NS)] = v[b * R + r];
    }
    __syncthreads();
}

// Forward transforms of NROWS rows of 2^LOGL values in LDS (natural order in and out; the
// caller synchronises before).
template <int LOGL, int NROWS, int LOGT, int P = 0>
__device__ __forceinline__ void fft_rows(float2 *buf, const float2 *tab, int t) {
    using FP = FftPasses<LOGL>;
    if constexpr (P < FP::N) {
        fft_pass<LOGL, NROWS, FP::log_radix(P), FP::log_ns(P), LOGT>(buf, tab, t);
        fft_rows<LOGL, NROWS, LOGT, P + 1>(buf, tab, t);
    }
}

// tab[m] = W_T^m = exp(-2 pi i m / T), m < T / 2 (T = 2^LOGT), from the float64-derived
// two-level table (each entry within ~1.5 ulp), built in `lohi` (128 values of LDS that are
// free until the call returns); synchronises before returning.
template <int LOGT>
__device__ __forceinline__ void fill_twiddles(float2 *tab, float2 *lohi, int t) {
    const TwiddleTable tw = build_twiddles(lohi, lohi + 64, LOGT, t, 256);
    __syncthreads();
    for (int m = t; m < (1 << (LOGT - 1)); m += 256) tab[m] = tw(m);
    __syncthreads();
}

// Stokes I of every candidate pair of every channel of a chunk (the gridder applies the
// membership test of B): the scattered visibility reads happen here, with one thread per
// (channel, pair).  The correlator can write the same values from its epilogue instead.
template <typename VT>
__device__ __forceinline__ void stokes_gather(const VT *__restrict__ vis, const int2 *__restrict__ pairs,
                                              int n_pairs, int n_ant, float2 *__restrict__ cvis, int c, int k) {
    if (k >= n_pairs) return;
    const int2 p = pairs[k];
    const size_t nprod = (size_t)(2 * n_ant) * (2 * n_ant + 1) / 2;
    cvis[(size_t)c * n_pairs + k] = stokes_i<VT>(vis + (size_t)c * nprod, p.x, p.y);
}

template <typename VT>
__global__ __launch_bounds__(256) void stokes_gather_kernel(const VT *__restrict__ vis, const int2 *__restrict__ pairs,
                                                            int n_pairs, int n_ant, float2 *__restrict__ cvis) {
    stokes_gather<VT>(vis, pairs, n_pairs, n_ant, cvis, blockIdx.y, blockIdx.x * 256 + threadIdx.x);
}

// Gridding without atomics.  A workgroup grids one band of R rows of the upper half (v >= 0) of
// the 2n x 2n Hermitian grid, each pair entering at +(u, v) with V and at -(u, v) with conj V
// where its footprint reaches those rows; every thread owns a fixed rectangle of GE cells of it
// (CPT consecutive columns x RPT rows) in registers and sums the baselines whose 8 x 8 kernel
// footprint covers it, then the band is transformed along u and the n kept columns are written
// as the band's tile of the intermediate: [channel][band][image column][R rows], n R complex
// values, one contiguous block per workgroup.  The band's items are sorted by signed x
// separation, hence by grid column for every channel (u is proportional to dx).
// Each staging round puts a run of them in LDS with their 8 + 8 separable kernel weights
// (evaluated once per baseline) and a table of the first staged baseline at or right of every
// grid column, so a thread's baselines are the contiguous range of those starting within 7
// columns left of its first column, and it applies them as val * wu (once per column) times wv
// (once per cell).  Each cell sums its baselines in list order, so the result is deterministic.
template <int LOGM, int GE>
struct GridShape {
    static constexpr int M = 1 << LOGM;
    static constexpr int CELLS = Tile<GE>::CELLS;
    static constexpr int R = CELLS / M;              // rows of a band
    static constexpr int NB = M / 2 / R;             // bands of the half plane
    static constexpr int RS = RowLayout<M>::RS;
    static constexpr int BUF = R * RS;               // LDS complex values of the band
    // owned columns per thread: 4 x 4 cells at M = 512 (measured 3.5% faster than 2 x 8 there),
    // else one column per 256 of M
    static constexpr int CPT = M == 512 ? 4 : (M >= 256 ? M / 256 : 1);
    static constexpr int COLT = M / CPT;             // threads across the columns
    static constexpr int RPT = R / (256 / COLT);     // owned rows per thread
    static constexpr int XMIN = -16, XMAX = M + 16;  // first-index table range
    static constexpr int NFIRST = XMAX - XMIN + 1;
    // staged weights per baseline: wu[0..7] and wv[0..7], each with zeros on both sides so a
    // thread reads its CPT (RPT) consecutive entries at any footprint offset without a test
    // (odd stride: the lanes of a wave read different baselines, so they fall in different banks)
    static constexpr int WU = 8 + 2 * (CPT - 1), WV = 8 + 2 * (RPT - 1), WSTRIDE = (WU + WV) | 1;
    // staged per baseline: first footprint cell (int2), value (float2), padded weights; at most
    // one per thread and round
    static constexpr int CAP0 = (BUF * (int)sizeof(float2) - NFIRST * 4) / (8 + 8 + WSTRIDE * 4);
    static constexpr int CAP = CAP0 < 256 ? CAP0 : 256;
    static_assert(CPT * RPT == GE, "GE cells per thread");
    static_assert(CAP >= 64, "staging room");
};

// What one thread loads for the baseline it stages in a round: its list item, the membership
// word of B, Stokes I and the antenna separation.
struct StageIn {
    int item = 0;
    unsigned word = 0;
    float2 val = make_float2(0.f, 0.f);
    double2 d = make_double2(0.0, 0.0);
};

__device__ __forceinline__ StageIn stage_load(int item, const float2 *__restrict__ cv_c, const double2 *__restrict__ dxy,
                                              const SetTest &bset, int c) {
    StageIn s;
    const int k = item >> 1;
    s.item = item;
    s.word = bset.bits[(size_t)c * bset.words + (k >> 5)];
    s.val = cv_c[k];
    s.d = dxy[k];
    return s;
}

template <int LOGM, int PREC, int GE>
__device__ __forceinline__ void grid_rows(const float2 *__restrict__ cvis, const double2 *__restrict__ dxy,
                                          const double *__restrict__ freq, const int *__restrict__ band_off,
                                          const int *__restrict__ band_items, int n_pairs, const SetTest &bset,
                                          float2 *__restrict__ inter, int band, int c, float2 *grid, float2 *tab,
                                          float &vscale) {
    using GS = GridShape<LOGM, GE>;
    constexpr int M = GS::M, R = GS::R, RS = GS::RS, CPT = GS::CPT, COLT = GS::COLT, RPT = GS::RPT, CAP = GS::CAP;
    constexpr int n_pix = M / 2;
    // staging view of the band's LDS
    int2 *s_g = reinterpret_cast<int2 *>(grid);                   // gu0, gv0: first footprint cell
    float2 *s_val = reinterpret_cast<float2 *>(s_g + CAP);         // Stokes I value
    float *s_w = reinterpret_cast<float *>(s_val + CAP);           // padded wu, then padded wv
    int *s_first = reinterpret_cast<int *>(s_w + GS::WSTRIDE * CAP);  // [x - XMIN]: first i with gu0 >= x

    const int t = threadIdx.x;
    const int row0 = M / 2 + band * R;  // bands cover the rows v >= 0 of the Hermitian grid
    const float2 *cv_c = cvis + (size_t)c * n_pairs;
    const int k_begin = band_off[band], k_end = band_off[band + 1];
    const int n_items = k_end - k_begin;
    const int n_rounds = (n_items + CAP - 1) / CAP;
    // Round rr stages list entries rr, rr + n_rounds, ... (sorted by column and spread over the
    // whole band, so every wave has work in every round); thread t stages entry t n_rounds + rr,
    // so its entries are contiguous.  The loads run ahead of their use: the entry two rounds
    // ahead and the staged data of the next round are in flight while a round is gridded.
    const int *my = band_items + k_begin + t * n_rounds;
    auto has = [&](int rr) { return rr < n_rounds && t * n_rounds + rr < n_items; };
    int it_nxt = has(1) ? my[1] : 0;
    StageIn cur;
    if (has(0)) cur = stage_load(my[0], cv_c, dxy, bset, c);
    fill_twiddles<LOGM>(tab, grid, t);  // (the band's LDS is free until staging)
    if constexpr (PREC == NBSI_PREC_FP16) {
        // Scale this workgroup's visibilities by a power of two so the largest |V_I| it grids
        // maps below 2^14: every FP16 product (kernel weights <= 1) stays finite.
        float *red = reinterpret_cast<float *>(grid);
        float mx = 0.f;
        for (int i = k_begin + t; i < k_end; i += 256) {
            const int k = band_items[i] >> 1;
            if (!bset(c, k)) continue;
            const float2 val = cv_c[k];
            mx = fmaxf(mx, fmaxf(fabsf(val.x), fabsf(val.y)));
        }
        red[t] = mx;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (t < s) red[t] = fmaxf(red[t], red[t + s]);
            __syncthreads();
        }
        if (t == 0) {
            int e2 = 0;
            frexpf(fmaxf(red[0], 1e-30f), &e2);
            vscale = ldexpf(1.f, 14 - e2);
        }
        __syncthreads();
    }
    const int col0 = (t % COLT) * CPT;
    const int rown = (t / COLT) * RPT;  // first owned row within the band
    float2 acc[CPT][RPT];
#pragma unroll
    for (int q = 0; q < CPT; q++)
#pragma unroll
        for (int r = 0; r < RPT; r++) acc[q][r] = make_float2(0.f, 0.f);

    // grid position u / du + M/2 with du = 1/4 wavelength; candidate pairs outside B at this
    // channel's frequency are staged with a zero value
    const double sc = freq[c] / C_LIGHT * 4.0;
    for (int rr = 0; rr < n_rounds; rr++) {
        const int nk = (n_items - rr + n_rounds - 1) / n_rounds;
        StageIn nxt;
        if (has(rr + 1)) nxt = stage_load(it_nxt, cv_c, dxy, bset, c);
        const int it_after = has(rr + 2) ? my[rr + 2] : 0;
        __syncthreads();  // the previous round's staging area is free
        if (has(rr)) {
            const int i = t;
            const int item = cur.item, k = item >> 1;
            float2 val = ((cur.word >> (k & 31)) & 1u) ? cur.val : make_float2(0.f, 0.f);
            // mirrored item: conj V at -(u, v)
            const double sgn = (item & 1) ? -sc : sc;
            if (item & 1) val.y = -val.y;
            if constexpr (PREC == NBSI_PREC_FP16) val = make_float2(val.x * vscale, val.y * vscale);
            const double cu = cur.d.x * sgn + (double)(M / 2), cvv = cur.d.y * sgn + (double)(M / 2);
            const double fu = floor(cu), fv = floor(cvv);
            s_g[i] = make_int2((int)fu - 3, (int)fv - 3);
            s_val[i] = val;
            const float ou = (float)(cu - fu), ov = (float)(cvv - fv);  // in [0, 1)
            // cell offsets from the baseline's grid position, in cells: (j - 3) - o
            float *w = s_w + i * GS::WSTRIDE;
#pragma unroll
            for (int q = 0; q < GS::WU; q++) {
                const int j = q - (CPT - 1);
                w[q] = (unsigned)j < 8u ? es_kernel_fast(((float)(j - 3) - ou) * 0.25f) : 0.f;
            }
#pragma unroll
            for (int q = 0; q < GS::WV; q++) {
                const int j = q - (RPT - 1);
                w[GS::WU + q] = (unsigned)j < 8u ? es_kernel_fast(((float)(j - 3) - ov) * 0.25f) : 0.f;
            }
        }
        for (int x = t; x < GS::NFIRST; x += 256) s_first[x] = nk;
        __syncthreads();
        // s_first[x - XMIN] = first staged i with gu0 >= x: baseline i owns the x in (gu0[i-1], gu0[i]]
        for (int i = t; i < nk; i += 256) {
            const int a = i == 0 ? GS::XMIN - 1 : min(max(s_g[i - 1].x, GS::XMIN - 1), GS::XMAX);
            const int b = min(max(s_g[i].x, GS::XMIN - 1), GS::XMAX);
            for (int x = a + 1; x <= b; x++) s_first[x - GS::XMIN] = i;
        }
        __syncthreads();
        // this thread's baselines: gu0 in [col0 - 7, col0 + CPT - 1]
        const int lo = s_first[col0 - 7 - GS::XMIN], hi = s_first[col0 + CPT - GS::XMIN];
        for (int i = lo; i < hi; i++) {
            const int2 g = s_g[i];
            const int dr0 = row0 + rown - g.y;  // footprint row of owned row 0
            if (dr0 + RPT <= 0 || dr0 >= 8) continue;
            const float2 val = s_val[i];
            // footprint column of owned column 0 is col0 - gu0 in [-(CPT-1), 7]; footprint row of
            // owned row 0 is dr0 in [-(RPT-1), 7]: both index the padded rows in range
            const float *wup = s_w + i * GS::WSTRIDE + (CPT - 1) + (col0 - g.x);
            const float *wvp = s_w + i * GS::WSTRIDE + GS::WU + (RPT - 1) + dr0;
            float wu[CPT], wv[RPT];
#pragma unroll
            for (int q = 0; q < CPT; q++) wu[q] = wup[q];
#pragma unroll
            for (int r = 0; r < RPT; r++) wv[r] = wvp[r];
            if constexpr (PREC == NBSI_PREC_FP32) {
#pragma unroll
                for (int q = 0; q < CPT; q++) {
                    const float2 vu = make_float2(val.x * wu[q], val.y * wu[q]);
#pragma unroll
                    for (int r = 0; r < RPT; r++) {
                        acc[q][r].x = fmaf(vu.x, wv[r], acc[q][r].x);
                        acc[q][r].y = fmaf(vu.y, wv[r], acc[q][r].y);
                    }
                }
            } else {
#pragma unroll
                for (int q = 0; q < CPT; q++)
#pragma unroll
                    for (int r = 0; r < RPT; r++) acc[q][r] = cadd(acc[q][r], grid_product<PREC>(val, wu[q], wv[r]));
            }
        }
        cur = nxt;
        it_nxt = it_after;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < CPT; q++)
#pragma unroll
        for (int r = 0; r < RPT; r++) grid[lds_at<M>(rown + r, col0 + q)] = acc[q][r];
    __syncthreads();
    fft_rows<LOGM, R, LOGM>(grid, tab, t);
    // keep image columns x: FFT index (x - n/2) mod M, times (-1)^(x - n/2); undo the FP16 scale;
    // the tile [x][R rows] is written as two rows per float4, contiguous over the workgroup
    const float unscale = (PREC == NBSI_PREC_FP16) ? 1.f / vscale : 1.f;
    constexpr int HALF = R / 2;
    float4 *dst = reinterpret_cast<float4 *>(inter + (size_t)c * n_pix * n_pix + (size_t)band * n_pix * R);
    for (int e = t; e < n_pix * HALF; e += 256) {
        const int x = e / HALF, lr = 2 * (e % HALF);
        const int xp = x - n_pix / 2;
        const int col = xp & (M - 1);
        const float sgn = (xp & 1) ? -unscale : unscale;
        const float2 f0 = grid[lds_at<M>(lr, col)], f1 = grid[lds_at<M>(lr + 1, col)];
        dst[e] = make_float4(f0.x * sgn, f0.y * sgn, f1.x * sgn, f1.y * sgn);
    }
}

// Row pass of the chunk's channels: XCD-aware order (all bands of a channel run on one XCD, so
// its Stokes I row is read into one L2 once).
template <int LOGM, int PREC, int GE>
__global__ __launch_bounds__(256) void grid_rows_kernel(const float2 *__restrict__ cvis, const double2 *__restrict__ dxy,
                                                        const double *__restrict__ freq, const int *__restrict__ band_off,
                                                        const int *__restrict__ band_items, int n_pairs, int n_chan,
                                                        SetTest bset, float2 *__restrict__ inter) {
    using GS = GridShape<LOGM, GE>;
    __shared__ float2 grid[GS::BUF];
    __shared__ float2 tab[1 << (LOGM - 1)];
    __shared__ float vscale;
    const int id = blockIdx.x, xcd = id & 7, slot = id >> 3;
    const int c = ((slot / GS::NB) << 3) + xcd, band = slot % GS::NB;
    if (c >= n_chan) return;
    grid_rows<LOGM, PREC, GE>(cvis, dxy, freq, band_off, band_items, n_pairs, bset, inter, band, c, grid, tab, vscale);
}

// Gridding of channel ranges of several sub-bands of one image size: task -> (job, channel,
// band), one workgroup per task.
template <int LOGM, int PREC, int GE>
__global__ __launch_bounds__(256) void grid_rows_batch_kernel(const ImgJob *__restrict__ jobs, int n_jobs,
                                                              int n_tasks) {
    using GS = GridShape<LOGM, GE>;
    __shared__ float2 grid[GS::BUF];
    __shared__ float2 tab[1 << (LOGM - 1)];
    __shared__ float vscale;
    const int task = blockIdx.x;
    if (task >= n_tasks) return;
    int j = 0;
    while (j + 1 < n_jobs && jobs[j + 1].rows_task0 <= task) j++;
    const ImgJob &jb = jobs[j];
    const int local = task - jb.rows_task0;
    const SetTest bset{jb.inb, (jb.n_pairs + 31) >> 5};
    grid_rows<LOGM, PREC, GE>(jb.cvis, jb.dxy, jb.freq, jb.band_off, jb.band_items, jb.n_pairs, bset, jb.inter,
                              local % GS::NB, local / GS::NB, grid, tab, vscale);
}

// Column pass.  After the row pass, column x of the Hermitian grid holds s[i] = H(x, i) for the
// stored rows i = n .. 2n - 1 (n = n_pix), and s[2n - i] = conj s[i], s[0] = 0 (that row is
// outside every footprint).  Its transform S[k] = sum_i s[i] w^(ik) (w = exp(-2 pi i / 2n)) is
// real, and one n-point transform gives it: with a[i] = s[i] + s[i + n] and
// b[i] = (s[i] - s[i + n]) w^i, i < n, the transform Z of z = a + i b has Z[m] = S[2m] + i S[2m+1].
// The image is S / 2 (the real part of the transform of the half-plane grid), times the kernel
// correction and 1 / |B|.  A workgroup takes NX consecutive columns: one contiguous block of
// NX x R values from every band's tile.
template <int LOGM, int GE>
struct ColShape {
    static constexpr int M = 1 << LOGM, N = M / 2, LOGN = LOGM - 1;
    static constexpr int NX = cols_per_band(GE, N);     // columns per workgroup
    static constexpr int RB = Tile<GE>::CELLS / M;       // rows per band of the row pass
    static constexpr int NBANDS = N / RB;
    static constexpr int RS = RowLayout<N>::RS;
    static constexpr int E = NX * N / 256;               // values per thread
    static constexpr int BUF = NX * RS;
    static constexpr int NXB = N / NX;                   // workgroups per channel
    static_assert(E >= 2 && E % 2 == 0 && RB >= 2, "float4 loads");
};

template <int LOGM, int GE>
__device__ __forceinline__ void grid_cols(const float2 *__restrict__ inter, const float *__restrict__ corr,
                                          const int *__restrict__ nb, float *__restrict__ img, int xb, int c,
                                          float2 *buf, float2 *tab, unsigned *__restrict__ flags) {
    using CS = ColShape<LOGM, GE>;
    constexpr int M = CS::M, n = CS::N, NX = CS::NX, RB = CS::RB, RS = CS::RS, E = CS::E;
    const int t = threadIdx.x;
    const int x0 = xb * NX;
    // every band's block of these columns: [xl][RB rows], two rows per float4
    const float4 *src = reinterpret_cast<const float4 *>(inter + (size_t)c * n * n);
    float4 r[E / 2];
#pragma unroll
    for (int q = 0; q < E / 2; q++) {
        const int e4 = t + 256 * q;
        const int b = e4 / (NX * RB / 2), w = e4 % (NX * RB / 2);
        r[q] = src[((size_t)b * n + x0) * (RB / 2) + w];
    }
    fill_twiddles<LOGM>(tab, buf, t);  // (buf is free until the tiles are stored)
#pragma unroll
    for (int q = 0; q < E / 2; q++) {
        const int e4 = t + 256 * q;
        const int b = e4 / (NX * RB / 2), w = e4 % (NX * RB / 2);
        const int xl = w / (RB / 2), lr = 2 * (w % (RB / 2));
        const int i = b * RB + lr;
        buf[lds_at<n>(xl, i)] = make_float2(r[q].x, r[q].y);
        buf[lds_at<n>(xl, i + 1)] = make_float2(r[q].z, r[q].w);
    }
    __syncthreads();
    float2 z[E];
#pragma unroll
    for (int q = 0; q < E; q++) {
        const int e = t + 256 * q;
        const int xl = e / n, i = e % n;
        const float2 hi = buf[lds_at<n>(xl, i)];  // s[i + n]
        float2 lo = make_float2(0.f, 0.f);
        if (i) {
            const float2 m = buf[lds_at<n>(xl, n - i)];  // s[i] = conj s[2n - i], stored at row n - i
            lo = make_float2(m.x, -m.y);
        }
        const float2 a = cadd(lo, hi);
        const float2 bb = cmul(make_float2(lo.x - hi.x, lo.y - hi.y), tab[i]);  // w^i = W_M^i
        z[q] = make_float2(a.x - bb.y, a.y + bb.x);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < E; q++) {
        const int e = t + 256 * q;
        buf[lds_at<n>(e / n, e % n)] = z[q];
    }
    __syncthreads();
    fft_rows<CS::LOGN, NX, LOGM>(buf, tab, t);
    const int cnt = nb[c];
    const float inv = cnt > 0 ? (float)(0.5 / (double)cnt) : 0.f;
    bool bad = false;
    for (int e = t; e < n * NX; e += 256) {
        const int xl = e % NX, y = e / NX;
        const int yp = y - n / 2;
        const int k = yp & (M - 1);
        const float2 f = buf[lds_at<n>(xl, k >> 1)];
        const float v = (k & 1) ? f.y : f.x;
        const float sgn = (yp & 1) ? -1.f : 1.f;
        const float o = v * sgn * corr[x0 + xl] * corr[y] * inv;
        bad |= !__builtin_isfinite(o);
        img[((size_t)c * n + y) * n + x0 + xl] = o;
    }
    flag_nonfinite(bad, flags);
}

// Column pass of the chunk's channels, in the row pass's XCD-aware order.
template <int LOGM, int GE>
__global__ __launch_bounds__(256) void grid_cols_kernel(const float2 *__restrict__ inter, int n_chan,
                                                        const float *__restrict__ corr, const int *__restrict__ nb,
                                                        float *__restrict__ img, unsigned *__restrict__ flags) {
    using CS = ColShape<LOGM, GE>;
    __shared__ float2 buf[CS::BUF];
    __shared__ float2 tab[1 << (LOGM - 1)];
    const int id = blockIdx.x, xcd = id & 7, slot = id >> 3;
    const int c = ((slot / CS::NXB) << 3) + xcd, xb = slot % CS::NXB;
    if (c >= n_chan) return;
    grid_cols<LOGM, GE>(inter, corr, nb, img, xb, c, buf, tab, flags);
}

template <int LOGM, int GE>
__global__ __launch_bounds__(256) void grid_cols_batch_kernel(const ImgJob *__restrict__ jobs, int n_jobs,
                                                              int n_tasks) {
    using CS = ColShape<LOGM, GE>;
    __shared__ float2 buf[CS::BUF];
    __shared__ float2 tab[1 << (LOGM - 1)];
    const int task = blockIdx.x;  // one workgroup per (job, channel, column band)
    if (task >= n_tasks) return;
    int j = 0;
    while (j + 1 < n_jobs && jobs[j + 1].cols_task0 <= task) j++;
    const ImgJob &jb = jobs[j];
    const int local = task - jb.cols_task0;
    grid_cols<LOGM, GE>(jb.inter, jb.corr, jb.nb, jb.img, local % CS::NXB, local / CS::NXB, buf, tab, jb.flags);
}

// Gather over channel ranges of several sub-bands: one workgroup per (job, channel, 256 pairs).
__global__ __launch_bounds__(256) void stokes_gather_batch_kernel(const ImgJob *__restrict__ jobs, int n_jobs,
                                                                  int n_tasks) {
    const int task = blockIdx.x;
    if (task >= n_tasks) return;
    int j = 0;
    while (j + 1 < n_jobs && jobs[j + 1].gather_task0 <= task) j++;
    const ImgJob &jb = jobs[j];
    const int local = task - jb.gather_task0;
    const int nblk = (jb.n_pairs + 255) / 256;
    stokes_gather<int2>(reinterpret_cast<const int2 *>(jb.vis), jb.pairs, jb.n_pairs, jb.n_ant, jb.cvis, local / nblk,
                        (local % nblk) * 256 + threadIdx.x);
}

}  // namespace

hipError_t launch_image_count(const nbsi_image_plan *p, hipStream_t st) {
    hipLaunchKernelGGL(count_kernel, dim3(p->n_chan), dim3(256), 0, st, p->d_xyz, p->d_freq, p->d_pairs,
                       p->n_pairs, p->method == NBSI_IMAGE_GRID ? p->n_pix : 0, p->uv_min, p->uv_max,
                       p->d_nb, p->d_inb);
    return hipGetLastError();
}

hipError_t launch_image_dft(const nbsi_image_plan *p, const void *vis, int vis_dtype, float *img,
                            hipStream_t st, unsigned *flags) {
    dim3 grid(p->n_pix, p->n_chan);
    if (vis_dtype == NBSI_VIS_I32)
        hipLaunchKernelGGL(dft_kernel<int2>, grid, dim3(256), 0, st, (const int2 *)vis, p->d_xyz, p->d_freq,
                           p->d_pairs, p->n_pairs, p->n_ant, p->n_pix, p->uv_min, p->uv_max, p->d_nb, img, flags);
    else
        hipLaunchKernelGGL(dft_kernel<float2>, grid, dim3(256), 0, st, (const float2 *)vis, p->d_xyz,
                           p->d_freq, p->d_pairs, p->n_pairs, p->n_ant, p->n_pix, p->uv_min, p->uv_max,
                           p->d_nb, img, flags);
    return hipGetLastError();
}

template <int LOGM, int GE>
static hipError_t launch_grid_m(const nbsi_image_plan *p, int precision, const float2 *cvis, float2 *inter, float *img,
                                hipStream_t st, unsigned *flags) {
    const int c8 = (p->n_chan + 7) / 8 * 8;  // XCD-aware order: eight channels per round of blocks
    const SetTest bset{p->d_inb, (p->n_pairs + 31) >> 5};
    const dim3 gr((unsigned)(GridShape<LOGM, GE>::NB * c8));
#define NBSI_ROWS(PR)                                                                                           \
    hipLaunchKernelGGL((grid_rows_kernel<LOGM, PR, GE>), gr, dim3(256), 0, st, cvis, p->d_dxy, p->d_freq,      \
                       p->d_band_off, p->d_band_items, p->n_pairs, p->n_chan, bset, inter)
    if (precision == NBSI_PREC_FP16) NBSI_ROWS(NBSI_PREC_FP16);
    else if (precision == NBSI_PREC_BF16) NBSI_ROWS(NBSI_PREC_BF16);
    else NBSI_ROWS(NBSI_PREC_FP32);
#undef NBSI_ROWS
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((grid_cols_kernel<LOGM, GE>), dim3((unsigned)(ColShape<LOGM, GE>::NXB * c8)), dim3(256), 0, st,
                       inter, p->n_chan, p->d_corr, p->d_nb, img, flags);
    return hipGetLastError();
}

template <int GE>
static hipError_t launch_grid_ge(const nbsi_image_plan *p, int precision, const float2 *cvis, float2 *inter, float *img,
                                 int log_m, hipStream_t st, unsigned *flags) {
    switch (log_m) {
        case 7: return launch_grid_m<7, GE>(p, precision, cvis, inter, img, st, flags);
        case 8: return launch_grid_m<8, GE>(p, precision, cvis, inter, img, st, flags);
        case 9: return launch_grid_m<9, GE>(p, precision, cvis, inter, img, st, flags);
        case 10: return launch_grid_m<10, GE>(p, precision, cvis, inter, img, st, flags);
        case 11: return launch_grid_m<11, GE>(p, precision, cvis, inter, img, st, flags);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_image_grid_stokes(const nbsi_image_plan *p, const float2 *cvis, int precision, float2 *inter,
                                    float *img, hipStream_t st, unsigned *flags) {
    const int log_m = 31 - __builtin_clz(2 * p->n_pix);
    return p->ge == 32 ? launch_grid_ge<32>(p, precision, cvis, inter, img, log_m, st, flags)
                       : launch_grid_ge<16>(p, precision, cvis, inter, img, log_m, st, flags);
}

hipError_t launch_image_grid(const nbsi_image_plan *p, const void *vis, int vis_dtype, int precision,
                             float2 *cvis, float2 *inter, float *img, hipStream_t st, unsigned *flags) {
    dim3 gg((p->n_pairs + 255) / 256, p->n_chan);
    if (vis_dtype == NBSI_VIS_I32)
        hipLaunchKernelGGL(stokes_gather_kernel<int2>, gg, dim3(256), 0, st, (const int2 *)vis, p->d_pairs,
                           p->n_pairs, p->n_ant, cvis);
    else
        hipLaunchKernelGGL(stokes_gather_kernel<float2>, gg, dim3(256), 0, st, (const float2 *)vis, p->d_pairs,
                           p->n_pairs, p->n_ant, cvis);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_image_grid_stokes(p, cvis, precision, inter, img, st, flags);
}

hipError_t launch_image_batch_gather(const ImgJob *d_jobs, int n_jobs, int n_tasks, hipStream_t st) {
    hipLaunchKernelGGL(stokes_gather_batch_kernel, dim3(n_tasks), dim3(256), 0, st, d_jobs, n_jobs, n_tasks);
    return hipGetLastError();
}

template <int GE>
static hipError_t launch_batch_rows_ge(const ImgJob *d_jobs, int n_jobs, int n_tasks, int log_m, int precision,
                                       hipStream_t st) {
#define NBSI_BR(LM, PR)                                                                                        \
    hipLaunchKernelGGL((grid_rows_batch_kernel<LM, PR, GE>), dim3(n_tasks), dim3(256), 0, st, d_jobs, n_jobs, \
                       n_tasks)
#define NBSI_BR_P(LM)                                                    \
    if (precision == NBSI_PREC_FP16) NBSI_BR(LM, NBSI_PREC_FP16);         \
    else if (precision == NBSI_PREC_BF16) NBSI_BR(LM, NBSI_PREC_BF16);    \
    else NBSI_BR(LM, NBSI_PREC_FP32)
    switch (log_m) {
        case 7: NBSI_BR_P(7); break;
        case 8: NBSI_BR_P(8); break;
        case 9: NBSI_BR_P(9); break;
        case 10: NBSI_BR_P(10); break;
        case 11: NBSI_BR_P(11); break;
        default: return hipErrorInvalidValue;
    }
#undef NBSI_BR_P
#undef NBSI_BR
    return hipGetLastError();
}

hipError_t launch_image_batch_rows(const ImgJob *d_jobs, int n_jobs, int n_tasks, int log_m, int precision, int ge,
                                   hipStream_t st) {
    return ge == 32 ? launch_batch_rows_ge<32>(d_jobs, n_jobs, n_tasks, log_m, precision, st)
                    : launch_batch_rows_ge<16>(d_jobs, n_jobs, n_tasks, log_m, precision, st);
}

template <int GE>
static hipError_t launch_batch_cols_ge(const ImgJob *d_jobs, int n_jobs, int n_tasks, int log_m, hipStream_t st) {
    switch (log_m) {
        case 7: hipLaunchKernelGGL((grid_cols_batch_kernel<7, GE>), dim3(n_tasks), dim3(256), 0, st, d_jobs, n_jobs, n_tasks); break;
        case 8: hipLaunchKernelGGL((grid_cols_batch_kernel<8, GE>), dim3(n_tasks), dim3(256), 0, st, d_jobs, n_jobs, n_tasks); break;
        case 9: hipLaunchKernelGGL((grid_cols_batch_kernel<9, GE>), dim3(n_tasks), dim3(256), 0, st, d_jobs, n_jobs, n_tasks); break;
        case 10: hipLaunchKernelGGL((grid_cols_batch_kernel<10, GE>), dim3(n_tasks), dim3(256), 0, st, d_jobs, n_jobs, n_tasks); break;
        case 11: hipLaunchKernelGGL((grid_cols_batch_kernel<11, GE>), dim3(n_tasks), dim3(256), 0, st, d_jobs, n_jobs, n_tasks); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_image_batch_cols(const ImgJob *d_jobs, int n_jobs, int n_tasks, int log_m, int ge, hipStream_t st) {
    return ge == 32 ? launch_batch_cols_ge<32>(d_jobs, n_jobs, n_tasks, log_m, st)
                    : launch_batch_cols_ge<16>(d_jobs, n_jobs, n_tasks, log_m, st);
}
