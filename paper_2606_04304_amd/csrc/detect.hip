// Narrowband detection pass over a spectral cube (the paper's Sec. 2.4, Stage I with the
// width-1 matched filter), gfx950.
//
// Per-pixel kernel: a workgroup stages the spectra of PPW neighbouring pixels in LDS (one
// read of the cube), and one wave per pixel computes the exact median and MAD by a wave-local
// selection (sampled brackets checked by exact counts, no atomics and no barriers; see
// wave_select), scores every channel and keeps threshold crossings that survive +-1 channel
// non-maximum suppression (ties keep the lower channel).  Candidates are appended with a
// global atomic counter and sorted afterwards by (y, x, c) with a bitonic network.
//
// Per-image mode first computes each channel image's median and MAD over the visible
// hemisphere (a histogram selection over the image in global memory, one block per channel),
// then runs the per-pixel kernel on the standardised values with only the spectral median
// removed.
#include "internal.h"

namespace {

constexpr float MAD_K = 1.482602218505602f;


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

__device__ __forceinline__ float wave_min_f(float v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = fminf(v, __shfl_xor(v, d, 64));
    return v;
}
__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
    return v;
}

// Bin of x in [lo, hi] split into 256 equal parts: non-decreasing in x, safe for a zero-width
// or denormal range (an infinite scale sends everything above lo to the last bin).
__device__ __forceinline__ int value_bin(float x, float lo, float scale) {
    const float t = (x - lo) * scale;
    return t >= 256.f ? 255 : (t > 0.f ? (int)t : 0);
}

// Block-wide sum / min / max over SEL_NT threads through `red` (SEL_NT / 64 slots of LDS); every
// thread gets the result.  Callers keep the calls uniform across the block.
constexpr int SEL_NT = 1024;
constexpr int SEL_NW = SEL_NT / 64;
constexpr int SEL_POOL = 1024;

__device__ __forceinline__ int block_sum(int v, int *red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    int s = 0;
#pragma unroll
    for (int q = 0; q < SEL_NW; q++) s += red[q];
    return s;
}
__device__ __forceinline__ float block_min_f(float v, float *red) {
    v = wave_min_f(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    float s = INFINITY;
#pragma unroll
    for (int q = 0; q < SEL_NW; q++) s = fminf(s, red[q]);
    return s;
}
__device__ __forceinline__ float block_max_f(float v, float *red) {
    v = wave_max_f(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    float s = -INFINITY;
#pragma unroll
    for (int q = 0; q < SEL_NW; q++) s = fmaxf(s, red[q]);
    return s;
}

// LDS of one block selection
struct SelLds {
    unsigned hist[4][256];  // four copies (by wave % 4) against atomic contention
    int cnt[256];           // bin totals
    float pool[SEL_POOL];
    int ired[SEL_NW];
    float fred[SEL_NW];
    int sel[4];             // selected bin, values below it, values in it, pool fill
    float res;              // the selected value
};

// The rank-th smallest (0-based) of the values a block of SEL_NT threads enumerates (each(f)
// calls f on every value the calling thread owns; exact order statistic).  Values are binned by value over the current range [lo, hi] into 256 LDS
// counters; the bin index is a non-decreasing function of the value, so the bin holding the
// rank-th value is found from the cumulative counts, and the range shrinks to that bin's own
// min and max until at most SEL_POOL values remain, which are ranked directly.
template <typename Each>
__device__ __forceinline__ float block_kth(Each each, int rank, SelLds &L) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    float lo = INFINITY, hi = -INFINITY;
    each([&](float x) __attribute__((always_inline)) {
        lo = fminf(lo, x);
        hi = fmaxf(hi, x);
    });
    lo = block_min_f(lo, L.fred);
    hi = block_max_f(hi, L.fred);
    int k = rank;
    for (int iter = 0; iter < 40; iter++) {
        if (!(hi > lo)) return lo;  // uniform: one value left in range
        const float scale = 256.f / (hi - lo);
        for (int e = t; e < 4 * 256; e += SEL_NT) (&L.hist[0][0])[e] = 0;
        __syncthreads();
        each([&](float x) __attribute__((always_inline)) {
            if (x >= lo && x <= hi) atomicAdd(&L.hist[w & 3][value_bin(x, lo, scale)], 1u);
        });
        __syncthreads();
        if (t < 256) L.cnt[t] = (int)(L.hist[0][t] + L.hist[1][t] + L.hist[2][t] + L.hist[3][t]);
        __syncthreads();
        // the bin holding rank k: threads 0..255 own one bin each (waves 0..3)
        if (t < 256) {
            const int cnt = L.cnt[t];
            const int incl = wave_inclusive_scan(cnt, lane);
            if (lane == 63) L.ired[w] = incl;
            L.pool[t] = __int_as_float(cnt);  // park the count until the wave totals are known
            L.pool[256 + t] = __int_as_float(incl);
        }
        __syncthreads();
        if (t < 256) {
            int base = 0;
            for (int q = 0; q < w; q++) base += L.ired[q];
            const int cnt = __float_as_int(L.pool[t]);
            const int incl = base + __float_as_int(L.pool[256 + t]);
            if (incl - cnt <= k && k < incl) {
                L.sel[0] = t;
                L.sel[1] = incl - cnt;
                L.sel[2] = cnt;
            }
        }
        if (t == 0) L.sel[3] = 0;
        __syncthreads();
        const int bsel = L.sel[0], below = L.sel[1], cnt_in = L.sel[2];
        // min / max of the selected bin, and (when small) its values into the pool
        float nlo = INFINITY, nhi = -INFINITY;
        each([&](float x) __attribute__((always_inline)) {
            if (x >= lo && x <= hi && value_bin(x, lo, scale) == bsel) {
                nlo = fminf(nlo, x);
                nhi = fmaxf(nhi, x);
                if (cnt_in <= SEL_POOL) L.pool[atomicAdd(&L.sel[3], 1)] = x;
            }
        });
        nlo = block_min_f(nlo, L.fred);  // (its barriers also order the pool writes)
        nhi = block_max_f(nhi, L.fred);
        k -= below;
        if (cnt_in <= SEL_POOL) {
            // exact rank within the pool: the pool value with k values below it (ties: any copy)
            for (int e = t; e < cnt_in; e += SEL_NT) {
                const float v = L.pool[e];
                int less = 0, eq = 0;
                for (int j = 0; j < cnt_in; j++) {
                    const float y = L.pool[j];
                    less += y < v;
                    eq += y == v;
                }
                if (less <= k && k < less + eq) L.res = v;  // every writer writes the same value
            }
            __syncthreads();
            const float r = L.res;
            __syncthreads();
            return r;
        }
        lo = nlo;
        hi = nhi;
    }
    return lo;
}

// Median of the n_valid values the block enumerates (mean of the central pair for even
// n_valid).
template <typename Each>
__device__ __forceinline__ float block_median(Each each, int n_valid, SelLds &L) {
    const float vlo = block_kth(each, (n_valid - 1) / 2, L);
    if (n_valid & 1) return vlo;
    // rank n_valid/2: vlo itself when more than n_valid/2 values are <= vlo, else the next
    // larger value
    int le = 0;
    float nxt = INFINITY;
    each([&](float x) __attribute__((always_inline)) {
        le += x <= vlo;
        if (x > vlo) nxt = fminf(nxt, x);
    });
    le = block_sum(le, L.ired);
    nxt = block_min_f(nxt, L.fred);
    const float vhi = (le >= n_valid / 2 + 1) ? vlo : nxt;
    return 0.5f * (vlo + vhi);
}

// A wave-uniform value moved to a scalar register (frees vector registers in the selection loops).
__device__ __forceinline__ float uniform_f(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ int uniform_i(int x) { return __builtin_amdgcn_readfirstlane(x); }

// The next float above / below a finite x (the bracket bounds around a dropped pivot value).
__device__ __forceinline__ float float_up(float x) {
    if (x == 0.f) return __int_as_float(1);  // smallest positive denormal
    const int b = __float_as_int(x);
    return __int_as_float(x > 0.f ? b + 1 : b - 1);
}
__device__ __forceinline__ float float_down(float x) { return -float_up(-x); }

// Ascending bitonic sort of one value per lane across the wave (64 values).
__device__ __forceinline__ float wave_sort64(float v, int lane) {
#pragma unroll
    for (int size = 2; size <= 64; size <<= 1)
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const float o = __shfl_xor(v, stride, 64);
            const bool keep_min = ((lane & stride) == 0) == ((lane & size) == 0);
            v = keep_min ? fminf(v, o) : fmaxf(v, o);
        }
    return v;
}

// Pseudo-random 32-bit hash of (i, round), for reservoir sampling.
__device__ __forceinline__ unsigned mix_hash(unsigned i, unsigned round) {
    unsigned h = i * 0x9E3779B1u + round * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    return h;
}

// The rank-th smallest (0-based) of val(i), i < n (finite values), for one wave, without
// atomics or barriers.  The wave keeps a bracket [lo, hi] of values known to hold the answer,
// with c_lt values below it and c_le values at or below its top (c_lt <= rank < c_le).  Each
// round sorts a sample of in-bracket values (one per lane, drawn from the entries l, l + 64, ...),
// takes the sample values D places either side of the rank's expected place as a candidate
// [a, b] (a single pivot value when the bracket did not shrink last round), and counts the data
// below a and at or below b: the rank then lies below a, in [a, b] or above b, and the bracket
// becomes that part.  The counting pass also keeps the first value of the lane's entries in
// [a, b], the next sample when the rank is there (the usual case); otherwise, and from round
// RESAMPLE_FROM on, a separate pass draws a uniform in-bracket sample by reservoir sampling,
// which keeps sorted or trending data from skewing the sample.  A pivot round always removes
// the pivot, so the loop ends; noise-like spectra need 3-4 rounds.  At most 64 values are left in
// the bracket then; they are gathered into `pool` (64 floats) and ranked exactly.
template <typename ValFn>
__device__ float wave_select(ValFn val, int n, int rank, float *pool, int lane) {
    constexpr int D = 8, RESAMPLE_FROM = 4;
    float lo = -INFINITY, hi = INFINITY;
    int c_lt = 0, c_le = n;
    float smp = lane < n ? val(lane) : INFINITY;  // this lane's sample of the bracket (+inf: none)
    bool pivot = false, resample = false;
    for (int round = 0; round < 2 * n + 2; round++) {
        const int m = c_le - c_lt;
        if (m <= 64 || lo == hi) break;
        if (resample || round >= RESAMPLE_FROM) {
            // uniform in-bracket value of this lane's entries (reservoir sampling)
            smp = INFINITY;
            int k = 0;
            for (int i = lane; i < n; i += 64) {
                const float x = val(i);
                if (x >= lo && x <= hi) {
                    k++;
                    if ((mix_hash((unsigned)i, (unsigned)round) >> 20) * (unsigned)k < 4096u) smp = x;
                }
            }
        }
        const float srt = wave_sort64(smp, lane);
        const int s_n = wave_sum(smp < INFINITY ? 1 : 0);  // >= 1: m > 64 values over 64 lanes
        const int p = min(s_n - 1, (int)(((long long)(rank - c_lt) * s_n) / m));
        float a, b;
        if (pivot) {
            a = b = __shfl(srt, p, 64);
        } else {
            a = p - D >= 0 ? __shfl(srt, p - D, 64) : lo;
            b = p + D < s_n ? __shfl(srt, p + D, 64) : hi;
            if (a == lo && b == hi) a = b = __shfl(srt, p, 64);
        }
        int n_lt = 0, n_le = 0;
        float s_in = INFINITY;
        for (int i = lane; i < n; i += 64) {
            const float x = val(i);
            n_lt += x < a;
            n_le += x <= b;
            s_in = (s_in == INFINITY && x >= a && x <= b) ? x : s_in;
        }
        n_lt = wave_sum(n_lt);
        n_le = wave_sum(n_le);
        resample = true;
        if (rank < n_lt) {  // below a
            hi = float_down(a);
            c_le = n_lt;
        } else if (rank >= n_le) {  // above b
            lo = float_up(b);
            c_lt = n_le;
        } else {  // in [a, b]
            if (a == b) return a;
            lo = a;
            hi = b;
            c_lt = n_lt;
            c_le = n_le;
            smp = s_in;
            resample = false;
        }
        pivot = c_le - c_lt == m;  // nothing left the bracket: split at a pivot next round
    }
    if (lo == hi) return lo;
    // at most 64 values in [lo, hi]: gather them and rank exactly
    int base = 0;
    for (int i0 = 0; i0 < n; i0 += 64) {
        const int i = i0 + lane;
        float x = 0.f;
        bool in = false;
        if (i < n) {
            x = val(i);
            in = x >= lo && x <= hi;
        }
        const unsigned long long bm = __ballot(in);
        if (in) pool[base + __popcll(bm & ((1ull << lane) - 1ull))] = x;
        base += __popcll(bm);
    }
    const int m = base;
    const int k = rank - c_lt;
    float mine = 0.f;
    bool hit = false;
    if (lane < m) {
        mine = pool[lane];
        int less = 0, eq = 0;
        for (int j = 0; j < m; j++) {
            const float y = pool[j];
            less += y < mine;
            eq += y == mine;
        }
        hit = less <= k && k < less + eq;
    }
    const unsigned long long hb = __ballot(hit);
    return __shfl(mine, hb ? (int)(__ffsll((long long)hb) - 1) : 0, 64);
}

// Median of val(i), i < n (finite values; mean of the central pair for even n), wave-local.
template <typename ValFn>
__device__ float wave_median_fast(ValFn val, int n, float *pool, int lane) {
    const float vlo = wave_select(val, n, (n - 1) / 2, pool, lane);
    if (n & 1) return vlo;
    int le = 0;
    float nxt = INFINITY;
    for (int i = lane; i < n; i += 64) {
        const float x = val(i);
        le += x <= vlo;
        if (x > vlo) nxt = fminf(nxt, x);
    }
    le = wave_sum(le);
    nxt = wave_min_f(nxt);
    const float vhi = (le >= n / 2 + 1) ? vlo : nxt;
    return 0.5f * (vlo + vhi);
}

// ---- spectra held in registers (n_chan <= 64 NR) ----
// Lane l of a wave holds channels l + 64 j, j < NR, of its pixel in v[j] (NaN past n_chan, which
// every comparison below treats as false).  The same algorithm as wave_select, with every pass
// over registers instead of LDS; a pass costs two compares and a select per held value on the
// vector unit, while the counts (popcounts of the compare masks) run on the scalar unit.
// The rank-th smallest held value, and the next one up when the last bracket shows it (NaN
// otherwise), for held values that are finite or NaN (NaN is never counted).
template <int NR>
__device__ float2 reg_select(const float (&v)[NR], int n, int rank, float *pool, int lane) {
    constexpr int D = 8, RESAMPLE_FROM = 4;
    float lo = -INFINITY, hi = INFINITY;
    int c_lt = 0, c_le = n;
    // first sample: lane l holds channel l + 64 (l mod NR), spread over the band (NaN past n);
    // the lanes that take register j form a constant mask
    float smp = INFINITY;
#pragma unroll
    for (int j = 0; j < NR; j++) {
        unsigned long long lanes_j = 0ull;
#pragma unroll
        for (int l = j % 64; l < 64; l += NR) lanes_j |= 1ull << l;
        smp = __builtin_amdgcn_inverse_ballot_w64(lanes_j) ? v[j] : smp;
    }
    smp = smp == smp ? smp : INFINITY;
    bool pivot = false, resample = false;
    for (int round = 0; round < 2 * n + 2; round++) {
        const int m = c_le - c_lt;
        if (m <= 64 || lo == hi) break;
        if (resample || round >= RESAMPLE_FROM) {
            smp = INFINITY;
            int k = 0;
#pragma unroll
            for (int j = 0; j < NR; j++) {
                const float x = v[j];
                if (x >= lo && x <= hi) {
                    k++;
                    if ((mix_hash((unsigned)(lane + 64 * j), (unsigned)round) >> 20) * (unsigned)k < 4096u) smp = x;
                }
            }
        }
        const float srt = wave_sort64(smp, lane);
        const int s_n = __popcll(__ballot(smp < INFINITY));
        const int p = min(s_n - 1, (int)(((long long)(rank - c_lt) * s_n) / m));
        float a, b;
        if (pivot) {
            a = b = __shfl(srt, p, 64);
        } else {
            a = p - D >= 0 ? __shfl(srt, p - D, 64) : lo;
            b = p + D < s_n ? __shfl(srt, p + D, 64) : hi;
            if (a == lo && b == hi) a = b = __shfl(srt, p, 64);
        }
        a = uniform_f(a);
        b = uniform_f(b);
        // count below a and at or below b (popcounts of the compare masks, on the scalar unit);
        // keep each lane's last held value in [a, b] (selected by the mask le & ~lt)
        int n_lt = 0, n_le = 0;
        float s_in = INFINITY;
#pragma unroll
        for (int j = 0; j < NR; j++) {
            const float x = v[j];
            const unsigned long long m_lt = __ballot(x < a), m_le = __ballot(x <= b);
            n_lt += __popcll(m_lt);
            n_le += __popcll(m_le);
            s_in = __builtin_amdgcn_inverse_ballot_w64(m_le & ~m_lt) ? x : s_in;
            // (an empty asm that takes s_in makes each select happen here: left alone, the
            // compiler defers the select chain and keeps every value's masks alive)
            asm volatile("" : "+v"(s_in));
        }
        // (the next sample is chosen before branching: were s_in needed on one path only, the
        // compiler would sink its selects there and keep every pass mask alive until then)
        const bool inside = rank >= n_lt && rank < n_le;
        smp = inside ? s_in : smp;
        resample = !inside;
        if (rank < n_lt) {
            hi = float_down(a);
            c_le = n_lt;
        } else if (rank >= n_le) {
            lo = float_up(b);
            c_lt = n_le;
        } else {
            if (a == b) return make_float2(a, rank + 1 < n_le ? a : NAN);
            lo = a;
            hi = b;
            c_lt = n_lt;
            c_le = n_le;
        }
        pivot = c_le - c_lt == m;
    }
    if (lo == hi) return make_float2(lo, rank + 1 < c_le ? lo : NAN);
    // at most 64 values remain in [lo, hi]: gathered one per lane through `pool`, sorted across
    // the wave, and read at the rank (and the next place, when it is in the bracket)
    int base = 0;
#pragma unroll
    for (int j = 0; j < NR; j++) {
        const float x = v[j];
        const bool in = x >= lo && x <= hi;
        const unsigned long long bm = __ballot(in);
        if (bm == 0ull) continue;  // (most registers hold none of them)
        if (in) pool[base + __popcll(bm & ((1ull << lane) - 1ull))] = x;
        base += __popcll(bm);
    }
    const int m = base;
    const float srt = wave_sort64(lane < m ? pool[lane] : INFINITY, lane);
    const int k = rank - c_lt;
    const float vk = __shfl(srt, k, 64), vk1 = __shfl(srt, min(k + 1, 63), 64);
    return make_float2(vk, k + 1 < m ? vk1 : NAN);
}

template <int NR>
__device__ float reg_median(const float (&v)[NR], int n, float *pool, int lane) {
    const float2 r = reg_select<NR>(v, n, (n - 1) / 2, pool, lane);
    if (n & 1) return r.x;
    float vhi = r.y;
    if (vhi != vhi) {  // the upper middle value was not in the last bracket: one more pass
        int le = 0;
        float nxt = INFINITY;
#pragma unroll
        for (int j = 0; j < NR; j++) {
            const float x = v[j];
            le += __popcll(__ballot(x <= r.x));
            nxt = fminf(nxt, x > r.x ? x : INFINITY);
        }
        nxt = wave_min_f(nxt);
        vhi = (le >= n / 2 + 1) ? r.x : nxt;
    }
    return 0.5f * (r.x + vhi);
}

// Per-pixel detection for spectra of up to 64 NR channels: a workgroup of REG_PX waves takes
// REG_PX adjacent pixels of one row; each staging round loads 1,024 channels x REG_PX pixels
// (4 REG_PX contiguous bytes per channel row) through an LDS tile, and every wave keeps its
// pixel's spectrum in registers, so the selections and the scoring run without LDS or barriers.
// Four-wave workgroups (four per CU at 128 registers, so staging reads run under other
// workgroups' selections) free their slot as soon as their slowest pixel is done: the rounds a
// selection needs vary from pixel to pixel, and eight-wave workgroups, which wait for the
// slowest of eight, were 5% slower (sixteen-wave ones 17%).
constexpr int REG_PX = 4;
constexpr int REG_LINE = 128 / (4 * REG_PX);  // workgroups that share a 128-byte line of a row
template <int NR>
__global__ __launch_bounds__(64 * REG_PX, 4) void detect_pixel_reg_kernel(const float *__restrict__ img, int n_chan, int n_pix,
                                                                int mode, const float2 *__restrict__ stats,
                                                                float thresh, float *__restrict__ snr_out,
                                                                nbsi_cand *__restrict__ cand, int cap,
                                                                int *__restrict__ counter, unsigned *__restrict__ flags) {
    constexpr int CH = 1024;              // channels per staging round (16 registers)
    constexpr int TPC = REG_PX / 4;       // threads per channel row segment (16 bytes each)
    constexpr int CPS = 64 * REG_PX / TPC;  // channels per load step (256)
    static_assert(NR % (CH / 64) == 0 && CH % CPS == 0, "staging rounds");
    __shared__ float tile[CH][REG_PX + 1];
    __shared__ float pool_all[REG_PX][64];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int groups_per_row = (n_pix + REG_PX - 1) / REG_PX;
    // XCD-aware order: workgroups are dealt to the 8 XCDs round robin, so the REG_LINE groups
    // that split each 128-byte line of a channel row go to blocks b, b + 8, ... of one XCD,
    // which run together and share the line in that XCD's L2
    constexpr int RUN = 8 * REG_LINE;
    const int nbr = (int)gridDim.x / RUN * RUN, b = blockIdx.x;
    const int grp = b < nbr ? (b / RUN) * RUN + (b & 7) * REG_LINE + ((b >> 3) % REG_LINE) : b;
    const int gy = grp / groups_per_row, gx0 = (grp % groups_per_row) * REG_PX;
    const size_t npix2 = (size_t)n_pix * n_pix;
    // staging: thread t loads pixels sp .. sp + 3 (16 bytes; n_pix is a multiple of 8) of
    // channels sc + CPS q
    const int sp = 4 * (t % TPC), sc = t / TPC;
    const bool col_ok = gx0 + sp < n_pix;
    const float *src = img + (size_t)gy * n_pix + gx0 + sp;
    // the loads of round k + 1 are issued before round k's tile is read back, so they are in
    // flight across its barrier
    auto load = [&](int k, float4 (&r)[CH / CPS]) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < CH / CPS; q++) {
            const int c = k * CH + sc + CPS * q;
            r[q] = (c < n_chan && col_ok) ? *reinterpret_cast<const float4 *>(src + (size_t)c * npix2)
                                          : make_float4(NAN, NAN, NAN, NAN);
        }
    };
    float v[NR];
    float4 r[CH / CPS];
    // pixels of the workgroup whose spectrum holds a non-finite value (bit = pixel), gathered
    // while staging
    __shared__ unsigned s_bad;
    if (t == 0) s_bad = 0u;
    load(0, r);
#pragma unroll
    for (int k = 0; k < NR / (CH / 64); k++) {
        __syncthreads();  // the previous round's tile has been read (and s_bad is cleared)
        unsigned bad_px = 0u;
#pragma unroll
        for (int q = 0; q < CH / CPS; q++) {
            const int c = k * CH + sc + CPS * q;
            float e[4] = {r[q].x, r[q].y, r[q].z, r[q].w};
            if (mode == NBSI_DETECT_PER_IMAGE && c < n_chan) {
                const float2 st = stats[c];
#pragma unroll
                for (int i = 0; i < 4; i++)  // (x * 0: non-finite stays non-finite)
                    e[i] = st.y > 0.f ? (e[i] - st.x) / st.y : e[i] * 0.f;
            }
#pragma unroll
            for (int i = 0; i < 4; i++) {
                tile[sc + CPS * q][sp + i] = e[i];
                if (c < n_chan && !__builtin_isfinite(e[i])) bad_px |= 1u << (sp + i);
            }
        }
        if (bad_px) atomicOr(&s_bad, bad_px);
        if (k + 1 < NR / (CH / 64)) load(k + 1, r);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < CH / 64; q++) v[(CH / 64) * k + q] = tile[lane + 64 * q][wave];
    }
    const int x = gx0 + wave, y = gy;
    if (x >= n_pix) return;  // no barriers below
    // a spectrum holding a non-finite value is not searched (wave-uniform: one pixel per wave)
    const bool finite = ((s_bad >> wave) & 1u) == 0u;
    const bool in_hor = in_horizon(x, y, n_pix);
    if (in_hor && !finite && lane == 0 && flags) atomicOr(flags, NBSI_FLAG_CUBE_NONFINITE);
    const bool active = in_hor && finite;
    float *pool = pool_all[wave];
    float scale = 1.f;
    bool ok = active;
    if (active) {
        const float med = reg_median<NR>(v, n_chan, pool, lane);
        // the deviations x - med replace the values (rounded as the score rounds them); for the
        // MAD their magnitudes, with the signs kept in a bit mask, so that both selections rank
        // values held in registers (a rank over |x - med| computed on the fly has the compiler
        // hoist all NR of them out of the selection rounds and spill)
        unsigned long long neg = 0ull;
#pragma unroll
        for (int j = 0; j < NR; j++) {
            const float d = v[j] - med;
            neg |= (unsigned long long)(d < 0.f) << j;
            v[j] = fabsf(d);  // (NaN past n_chan stays NaN)
        }
        if (mode == NBSI_DETECT_PER_PIXEL) {
            const float mad = reg_median<NR>(v, n_chan, pool, lane);
            scale = MAD_K * mad;
            ok = mad > 0.f;
        }
#pragma unroll
        for (int j = 0; j < NR; j++) v[j] = ((neg >> j) & 1ull) ? -v[j] : v[j];
    }
    // SNR = (x - med) / scale as a product with the float32 reciprocal; neighbours along
    // frequency come from the adjacent lane (channel c +- 1), across register rows at lanes 0/63
    const float inv = ok ? 1.f / scale : 0.f;
#pragma unroll
    for (int j = 0; j < NR; j++) {
        const int c = lane + 64 * j;
        const float xv = v[j];  // x - med
        const float z = ok ? xv * inv : 0.f;
        if (snr_out && c < n_chan) snr_out[(size_t)c * npix2 + (size_t)y * n_pix + x] = z;
        const bool hit = ok && c < n_chan && z >= thresh;
        // the neighbours are fetched (with every lane taking part) only when a lane crosses
        if (__ballot(hit) == 0ull) continue;
        const float up = __shfl_up(xv, 1, 64), dn = __shfl_down(xv, 1, 64);
        const float prev_row = j > 0 ? __shfl(v[j > 0 ? j - 1 : 0], 63, 64) : 0.f;
        const float next_row = j + 1 < NR ? __shfl(v[j + 1 < NR ? j + 1 : j], 0, 64) : 0.f;
        if (!hit) continue;
        const float xl = lane > 0 ? up : prev_row, xr = lane < 63 ? dn : next_row;
        if (c > 0 && !(z > xl * inv)) continue;
        if (c + 1 < n_chan && !(z >= xr * inv)) continue;
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

// stats: per-channel (median, k * MAD) for PER_IMAGE mode, else unused.
template <int PPW>
__global__ __launch_bounds__(64 * PPW) void detect_pixel_kernel(
    const float *__restrict__ img, int n_chan, int n_pix, int mode, const float2 *__restrict__ stats,
    float thresh, float *__restrict__ snr_out, nbsi_cand *__restrict__ cand, int cap, int *__restrict__ counter,
    int n_groups, unsigned *__restrict__ flags) {
    extern __shared__ float spec[];  // [PPW][n_chan]
    __shared__ float pool_all[PPW][64];
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
                v = st.y > 0.f ? (v - st.x) / st.y : v * 0.f;  // (v * 0: non-finite stays non-finite)
            }
        }
        spec[pl * n_chan + c] = v;
    }
    __syncthreads();
    const int x = gx0 + wave, y = gy;
    float *s = spec + wave * n_chan;
    // a spectrum holding a non-finite value is not searched (wave-uniform: one pixel per wave)
    bool bad = false;
    for (int c = lane; c < n_chan; c += 64) bad |= !__builtin_isfinite(s[c]);
    const bool finite = __ballot(bad) == 0ull;
    const bool in_hor = grp_ok && in_horizon(x, y, n_pix);
    if (in_hor && !finite && lane == 0 && flags) atomicOr(flags, NBSI_FLAG_CUBE_NONFINITE);
    const bool active = in_hor && finite;
    float *pool = pool_all[wave];
    auto val_x = [&](int i) { return s[i]; };
    const float med = finite ? wave_median_fast(val_x, n_chan, pool, lane) : 0.f;
    float scale = 1.f;  // SNR = (x - med) / scale
    bool ok = active;
    if (mode == NBSI_DETECT_PER_PIXEL && finite) {
        auto val_d = [&](int i) { return fabsf(s[i] - med); };
        const float mad = wave_median_fast(val_d, n_chan, pool, lane);
        scale = MAD_K * mad;
        ok = ok && mad > 0.f;
    }
    // SNR = (x - med) / scale, applied as a product with the float32 reciprocal (within an ulp of
    // the quotient; the same form scores neighbours for the suppression test)
    const float inv = ok ? 1.f / scale : 0.f;
    for (int c = lane; c < n_chan; c += 64) {
        const float z = ok ? (s[c] - med) * inv : 0.f;
        if (snr_out && grp_ok) snr_out[(size_t)c * npix2 + (size_t)y * n_pix + x] = z;
        if (!ok || z < thresh) continue;
        if (c > 0 && !(z > (s[c - 1] - med) * inv)) continue;
        if (c + 1 < n_chan && !(z >= (s[c + 1] - med) * inv)) continue;
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

// Per-channel median and k*MAD over the visible hemisphere (PER_IMAGE mode), one block of SEL_NT
// threads per channel image.  Thread t owns column x = t % n_pix and the rows
// y = y_lo(x) + t / n_pix, + G, ... (G = SEL_NT / n_pix row groups; for n_pix > SEL_NT a thread
// owns several columns) inside the hemisphere, whose extent in each column is an integer square
// root: coalesced row reads, no masking.  Up to 256 x 256 pixels a thread owns at most 64
// values, which are read once and kept on chip (32 in registers, the rest in LDS), so every pass
// of the selection runs from there; larger images are re-read each pass with eight loads in
// flight (the passes of many channels at once do not fit the caches).
__device__ __forceinline__ int isqrt_floor(int q) {  // largest r >= 0 with r * r <= q (q >= 0)
    int r = (int)sqrtf((float)q);
    while (r * r > q) r--;
    while ((r + 1) * (r + 1) <= q) r++;
    return r;
}

constexpr int STATS_VR = 32;  // values per thread in registers (n_pix <= 256)
constexpr int STATS_VL = 32;  // values per thread in LDS, [j][thread] (conflict-free rows)

template <bool ONCHIP>
__global__ __launch_bounds__(SEL_NT) void image_stats_kernel(const float *__restrict__ img, int n_pix,
                                                             float2 *__restrict__ stats) {
    __shared__ SelLds L;
    __shared__ float s_v[ONCHIP ? STATS_VL * SEL_NT : 1];
    const int c = blockIdx.x, t = threadIdx.x;
    const float *im = img + (size_t)c * n_pix * n_pix;
    const int h = n_pix / 2;
    const int G = n_pix <= SEL_NT ? SEL_NT / n_pix : 1;  // row groups
    const int g = n_pix <= SEL_NT ? t / n_pix : 0;
    const bool on = g < G;
    const int x0 = n_pix <= SEL_NT ? t % n_pix : t;
    // rows y0 + g, + G, ... <= y1 of column x in the hemisphere:
    // (x - h)^2 + (y - h)^2 < h^2  <=>  |y - h| <= isqrt(h^2 - (x - h)^2 - 1)
    auto rows = [&](int x, int &y0, int &y1) __attribute__((always_inline)) {
        const int q = h * h - (x - h) * (x - h);
        if (q <= 0) {
            y0 = 1;
            y1 = 0;
            return;
        }
        const int r = isqrt_floor(q - 1);
        y0 = h - r + g;
        y1 = h + r;
    };
    float v[ONCHIP ? STATS_VR : 1];
    int nv = 0;
    if constexpr (ONCHIP) {
        // n_pix <= 256: one column, at most ceil(n_pix / G) <= 64 rows
        int y0 = 1, y1 = 0;
        if (on) rows(x0, y0, y1);
        nv = y1 >= y0 ? (y1 - y0) / G + 1 : 0;
#pragma unroll
        for (int j = 0; j < STATS_VR; j++) v[j] = j < nv ? im[(size_t)(y0 + j * G) * n_pix + x0] : 0.f;
#pragma unroll
        for (int j = 0; j < STATS_VL; j++) {
            const int jj = STATS_VR + j;
            s_v[j * SEL_NT + t] = jj < nv ? im[(size_t)(y0 + jj * G) * n_pix + x0] : 0.f;
        }
        // (the selection's first block reduction orders these LDS writes before any read)
    }
    // every pass visits the finite values only (non-finite pixels take no part in the statistics)
    auto visit = [&](auto f) __attribute__((always_inline)) {
        if constexpr (ONCHIP) {
#pragma unroll
            for (int j = 0; j < STATS_VR; j++)
                if (j < nv && __builtin_isfinite(v[j])) f(v[j]);
            for (int j = 0; j < nv - STATS_VR; j++) {
                const float u = s_v[j * SEL_NT + t];
                if (__builtin_isfinite(u)) f(u);
            }
        } else {
            if (!on) return;
            for (int x = x0; x < n_pix; x += SEL_NT) {
                int y0, y1;
                rows(x, y0, y1);
                int y = y0;
                for (; y + 7 * G <= y1; y += 8 * G) {
                    float u[8];
#pragma unroll
                    for (int k = 0; k < 8; k++) u[k] = im[(size_t)(y + k * G) * n_pix + x];
#pragma unroll
                    for (int k = 0; k < 8; k++)
                        if (__builtin_isfinite(u[k])) f(u[k]);
                }
                for (; y <= y1; y += G) {
                    const float u1 = im[(size_t)y * n_pix + x];
                    if (__builtin_isfinite(u1)) f(u1);
                }
            }
        }
    };
    int n_in = 0;
    visit([&](float) __attribute__((always_inline)) { n_in++; });
    n_in = block_sum(n_in, L.ired);
    if (n_in == 0) {  // no finite pixel in this channel image (uniform)
        if (t == 0) stats[c] = make_float2(0.f, 0.f);
        return;
    }
    const float med = block_median([&](auto f) __attribute__((always_inline)) { visit(f); }, n_in, L);
    const float mad = block_median(
        [&](auto f) __attribute__((always_inline)) {
            visit([&](float x) __attribute__((always_inline)) { f(fabsf(x - med)); });
        },
        n_in, L);
    if (t == 0) stats[c] = make_float2(med, MAD_K * mad);
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

// The same bitonic network for at most SORT1_MAX candidates in one workgroup: keys in LDS, a
// barrier between steps (each pair (i, i ^ j) is handled by the thread of its lower index), and
// the gather of the sorted records.  One launch instead of one per step.
constexpr int SORT1_MAX = 4096;
__global__ __launch_bounds__(1024) void sort_small_kernel(const nbsi_cand *__restrict__ cand, int n, int n_pow2,
                                                          int n_chan, int n_pix, int n_out,
                                                          nbsi_cand *__restrict__ out) {
    __shared__ unsigned long long s[SORT1_MAX];
    const int t = threadIdx.x;
    for (int i = t; i < n_pow2; i += 1024)
        s[i] = (i < n) ? ((cand_key(cand[i], n_chan, n_pix) << 24) | (unsigned long long)i) : ~0ull;
    __syncthreads();
    for (int k = 2; k <= n_pow2; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = t; i < n_pow2; i += 1024) {
                const int p = i ^ j;
                if (p > i) {
                    const unsigned long long a = s[i], b = s[p];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        s[i] = b;
                        s[p] = a;
                    }
                }
            }
            __syncthreads();
        }
    for (int i = t; i < n_out; i += 1024) out[i] = cand[(int)(s[i] & 0xffffffull)];
}

// The small sort with the count read on the device: n = *counter candidates (when n <= cap and
// n <= SORT1_MAX; otherwise the host sorts once it has read n), the first min(n, n_out) of them
// written to out in (y, x, c) order.
__global__ __launch_bounds__(1024) void sort_small_dev_kernel(const nbsi_cand *__restrict__ cand,
                                                              const int *__restrict__ counter, int cap, int n_chan,
                                                              int n_pix, int n_out, nbsi_cand *__restrict__ out) {
    __shared__ unsigned long long s[SORT1_MAX];
    const int n = *counter;
    if (n <= 0 || n > cap || n > SORT1_MAX) return;
    int n_pow2 = 1;
    while (n_pow2 < n) n_pow2 <<= 1;
    const int t = threadIdx.x;
    for (int i = t; i < n_pow2; i += 1024)
        s[i] = (i < n) ? ((cand_key(cand[i], n_chan, n_pix) << 24) | (unsigned long long)i) : ~0ull;
    __syncthreads();
    for (int k = 2; k <= n_pow2; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = t; i < n_pow2; i += 1024) {
                const int p = i ^ j;
                if (p > i) {
                    const unsigned long long a = s[i], b = s[p];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        s[i] = b;
                        s[p] = a;
                    }
                }
            }
            __syncthreads();
        }
    const int m = min(n, n_out);
    for (int i = t; i < m; i += 1024) out[i] = cand[(int)(s[i] & 0xffffffull)];
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
    if (n_pix <= 256)
        hipLaunchKernelGGL(image_stats_kernel<true>, dim3(n_chan), dim3(SEL_NT), 0, st, img, n_pix,
                           reinterpret_cast<float2 *>(stats));
    else
        hipLaunchKernelGGL(image_stats_kernel<false>, dim3(n_chan), dim3(SEL_NT), 0, st, img, n_pix,
                           reinterpret_cast<float2 *>(stats));
    return hipGetLastError();
}

hipError_t launch_detect_scan(const float *img, int n_chan, int n_pix, int mode, const float *stats,
                              float thresh, float *snr, nbsi_cand *cand, int cap, int *counter,
                              hipStream_t st, unsigned *flags) {
    const float2 *s2 = reinterpret_cast<const float2 *>(stats);
    if (n_chan <= 64 * 64) {
        const int n_blocks = n_pix * ((n_pix + REG_PX - 1) / REG_PX);
        hipLaunchKernelGGL(detect_pixel_reg_kernel<64>, dim3(n_blocks), dim3(64 * REG_PX), 0, st, img, n_chan, n_pix,
                           mode, s2, thresh, snr, cand, cap, counter, flags);
        return hipGetLastError();
    }
    const int ppw = detect_ppw(n_chan);
    const int n_groups = n_pix * n_pix / ppw;
    // grid covers every group id produced by the XCD-aware mapping (blocks of 64 groups)
    const int n_blocks = ((n_groups + 63) / 64) * 64;
    const size_t lds = (size_t)ppw * n_chan * sizeof(float);
    // the staged spectra may exceed the default 64 KiB of dynamic LDS (gfx950 has 160 KiB)
    hipError_t ea = hipSuccess;
    if (ppw == 4) ea = hipFuncSetAttribute((const void *)detect_pixel_kernel<4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    else if (ppw == 2) ea = hipFuncSetAttribute((const void *)detect_pixel_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    else ea = hipFuncSetAttribute((const void *)detect_pixel_kernel<1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ea != hipSuccess) return ea;
    switch (ppw) {
        case 4:
            hipLaunchKernelGGL(detect_pixel_kernel<4>, dim3(n_blocks), dim3(256), lds, st, img, n_chan, n_pix, mode,
                               s2, thresh, snr, cand, cap, counter, n_groups, flags);
            break;
        case 2:
            hipLaunchKernelGGL(detect_pixel_kernel<2>, dim3(n_blocks), dim3(128), lds, st, img, n_chan, n_pix, mode,
                               s2, thresh, snr, cand, cap, counter, n_groups, flags);
            break;
        default:
            hipLaunchKernelGGL(detect_pixel_kernel<1>, dim3(n_blocks), dim3(64), lds, st, img, n_chan, n_pix, mode,
                               s2, thresh, snr, cand, cap, counter, n_groups, flags);
    }
    return hipGetLastError();
}

hipError_t launch_detect_sort_small_dev(const nbsi_cand *cand, const int *counter, int cap, int n_chan, int n_pix,
                                       nbsi_cand *out, int n_out, hipStream_t st) {
    if (n_out <= 0) return hipSuccess;
    hipLaunchKernelGGL(sort_small_dev_kernel, dim3(1), dim3(1024), 0, st, cand, counter, cap, n_chan, n_pix, n_out,
                       out);
    return hipGetLastError();
}

int detect_sort_small_max() { return SORT1_MAX; }

hipError_t launch_detect_sort(nbsi_cand *cand, int n, unsigned long long *keys, int n_chan, int n_pix,
                              nbsi_cand *out, int n_out, hipStream_t st) {
    if (n <= 0 || n_out <= 0) return hipSuccess;
    int n_pow2 = 1;
    while (n_pow2 < n) n_pow2 <<= 1;
    if (n_pow2 <= SORT1_MAX) {
        hipLaunchKernelGGL(sort_small_kernel, dim3(1), dim3(1024), 0, st, cand, n, n_pow2, n_chan, n_pix,
                           n_out <= n ? n_out : n, out);
        return hipGetLastError();
    }
    const int blocks = (n_pow2 + 255) / 256;
    hipLaunchKernelGGL(sort_keys_kernel, dim3(blocks), dim3(256), 0, st, cand, n, n_pow2, n_chan, n_pix, keys);
    for (int k = 2; k <= n_pow2; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1)
            hipLaunchKernelGGL(bitonic_step_kernel, dim3(blocks), dim3(256), 0, st, keys, n_pow2, j, k);
    hipLaunchKernelGGL(gather_sorted_kernel, dim3((n_out + 255) / 256), dim3(256), 0, st, keys, cand, n_out, out);
    return hipGetLastError();
}
