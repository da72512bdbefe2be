// Full cross-correlation (the paper's Sec. 2.1 X-engine) on gfx950 matrix cores.
//
// For one channel, stack the spectra as a real int8 matrix Y with 2 n_in rows (row 2i = Re q_i,
// row 2i+1 = Im q_i) and n_spec columns, and form the Gram matrix G = Y Y^T with
// v_mfma_i32_32x32x32_i8 (int32 accumulation, exact).  Every 2x2 block of G is one visibility:
//     Re V_ij = G[2i, 2j] + G[2i+1, 2j+1],   Im V_ij = G[2i+1, 2j] - G[2i, 2j+1]
// so no int8 value is ever negated (-128 is safe) and all four products of a block are useful.
// Only lower-triangle blocks of G are computed.
//
// Tiling: a workgroup (4 waves) owns a 128 x 128 block of G (64 x 64 visibilities) and loops
// over K = n_spec in 64-byte LDS stages; each wave owns 64 x 64 of G (2 x 2 MFMA tiles).
// The epilogue swaps accumulators with the neighbouring lane (DPP) to assemble complex
// visibilities and writes packed-triangle rows of 16 consecutive baselines (128 B) per lane
// group.  Block index -> (channel, tile pair) keeps every tile pair of a channel on one XCD so
// partial cache lines at tile edges merge in that XCD's L2.
#include "internal.h"

#include <algorithm>
#include <mutex>
#include <vector>

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

namespace {

constexpr int TILE = 128;        // G rows / cols per workgroup tile (FP32 path)
constexpr int TILE_I8 = 128;     // G rows / cols per workgroup tile of the int8 tiled kernel
constexpr int KC = 64;           // K bytes per LDS stage
constexpr int LDS_STRIDE = KC + 16;  // padded row stride (bytes): 16 rows of a b128 read hit 64 distinct banks

__device__ __forceinline__ void tile_pair(int pair, int &I, int &J) {
    int a = (int)((sqrtf(8.f * (float)pair + 1.f) - 1.f) * 0.5f);
    while ((a + 1) * (a + 2) / 2 <= pair) a++;
    while (a * (a + 1) / 2 > pair) a--;
    I = a;
    J = pair - a * (a + 1) / 2;
}

// One K stage of rows [r0, r0 + TILE_I8) x bytes [k0, k0 + KC) of Y (row stride ldy bytes), zero past
// T and past the last row, as STAGE_VECS 16-byte vectors per thread: loaded into registers one
// stage ahead, then stored to LDS.  Rows whose stride is a multiple of 16 bytes (the library
// repacks the others before a single-band launch) take whole-vector loads; other strides fall back
// to byte loads.
constexpr int STAGE_VECS = TILE_I8 * (KC / 16) / 256;
template <bool VEC>  // the row stride is a multiple of 16 bytes
__device__ __forceinline__ void load_stage(v4i (&v)[STAGE_VECS], const int8_t *__restrict__ Y, int rows, int T,
                                           int ldy, int r0, int k0, int t) {
#pragma unroll
    for (int i = 0; i < STAGE_VECS; i++) {
        const int e = t + 256 * i;
        const int rl = e / (KC / 16), vq = e % (KC / 16);
        const int r = r0 + rl, k = k0 + vq * 16;
        v4i val = {0, 0, 0, 0};
        if (r < rows && k < T) {
            const int8_t *src = Y + (size_t)r * ldy + k;
            if constexpr (VEC) {  // k + 16 <= ldy: bytes T .. ldy - 1 are the repacked zeros
                val = *reinterpret_cast<const v4i *>(src);
            } else {
                int8_t tmp[16];
#pragma unroll
                for (int b = 0; b < 16; b++) tmp[b] = (k + b < T) ? src[b] : (int8_t)0;
                val = *reinterpret_cast<v4i *>(tmp);
            }
        }
        v[i] = val;
    }
}

__device__ __forceinline__ void store_stage(int8_t *s, const v4i (&v)[STAGE_VECS], int t) {
#pragma unroll
    for (int i = 0; i < STAGE_VECS; i++) {
        const int e = t + 256 * i;
        const int rl = e / (KC / 16), vq = e % (KC / 16);
        *reinterpret_cast<v4i *>(s + rl * LDS_STRIDE + vq * 16) = v[i];
    }
}

__device__ __forceinline__ int swap_lanes(int x) {
    // quad_perm [1, 0, 3, 2]: exchange with the neighbouring lane
    return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, true);
}

// The Stokes-I mask and first index of the 8 x 8 antenna block of 32 x 32 tile (R0, C0) of G,
// as wave-uniform (scalar) values; zero when there is no Stokes-I output.
struct BlockStokes {
    unsigned long long mask = 0;
    int base = 0;
};
// The table is read only during the launch: reading it through the constant address space lets
// these uniform loads go to the scalar unit, so they never wait behind the wave's pending
// visibility stores (a vector load would, as the vector memory counter is shared by both).
typedef __attribute__((address_space(4))) const unsigned long long *const_u64_ptr;
typedef __attribute__((address_space(4))) const int *const_i32_ptr;
__device__ __forceinline__ BlockStokes block_stokes(const StokesOut &so, int R0, int C0) {
    BlockStokes r;
    if (so.out) {
        const int rb = R0 >> 5, cb = C0 >> 5;
        const int t = __builtin_amdgcn_readfirstlane(rb * (rb + 1) / 2 + cb);
        r.mask = ((const_u64_ptr)so.mask)[t];
        r.base = ((const_i32_ptr)so.base)[t];
    }
    return r;
}

// Calibration applied in the epilogue: w[i - r0] (rows) and w[j - c0] (columns) are LDS copies of
// channel c's complex correction factors; V'_ij = w_i V_ij conj(w_j) is written as float32 in
// place of the int32 visibility.  Null: plain int32 output.
struct CalIn {
    const float2 *wr = nullptr;
    int r0 = 0;
    const float2 *wc = nullptr;
    int c0 = 0;
};

// Combine a 32 x 32 tile of G (rows R0.., cols C0.., both even) into visibilities and store;
// with a Stokes-I output, also (V_XX + V_YY) / 2 of the block's candidate pairs of channel c.
// Lane l holds input row R0/2 + 4 qq + 2 (l / 32) + (l & 1) and input column C0/2 + (l % 32) / 2,
// so for a quad of lanes 4m .. 4m+3 the XX visibility of antenna pair (A, B) sits in lane 4m
// (inputs 2A, 2B) and the YY one in lane 4m+3 (inputs 2A+1, 2B+1); within the 8 x 8 antenna
// block, A % 8 = 2 qq + l / 32 and B % 8 = (l % 32) / 4.
// stage (optional): write the visibilities to an LDS tile instead, element (ia - stage_r0,
// b - stage_c0) at stage[(ia - stage_r0) * VIS_LDS_STRIDE + b - stage_c0] (rows outside the packed
// triangle included; the row writer skips them).
constexpr int VIS_LDS_STRIDE = 72;  // int2 per staged row: 4 rows of a store fall in different banks
__device__ __forceinline__ void store_tile_i32(const v16i &a, int R0, int C0, int lane, int n_in,
                                               int2 *__restrict__ vc, const StokesOut &so, int c,
                                               const BlockStokes &bs, bool small_sums, const CalIn &cal,
                                               int2 *stage = nullptr, int stage_r0 = 0, int stage_c0 = 0) {
    int par[16];
#pragma unroll
    for (int r = 0; r < 16; r++) par[r] = swap_lanes(a[r]);
    const int p = lane & 1, h = lane >> 5, cl = lane & 31;
    const int b = (C0 >> 1) + (cl >> 1);
#pragma unroll
    for (int qq = 0; qq < 4; qq++) {
        const int ia = (R0 >> 1) + 4 * qq + 2 * h + p;
        int re, im;
        if (p == 0) {  // column 2b: own rows 2a, 2a+1 at regs 4qq, 4qq+1
            re = a[4 * qq] + par[4 * qq + 1];
            im = a[4 * qq + 1] - par[4 * qq];
        } else {       // column 2b+1: rows 2a, 2a+1 at regs 4qq+2, 4qq+3
            re = par[4 * qq + 2] + a[4 * qq + 3];
            im = par[4 * qq + 3] - a[4 * qq + 2];
        }
        if (stage || (ia < n_in && b <= ia)) {
            int2 out = make_int2(re, im);
            if (cal.wr) {
                const float2 wi = cal.wr[ia - cal.r0], wj = cal.wc[b - cal.c0];
                const float vr = (float)re, vi = (float)im;
                const float tr = wi.x * vr - wi.y * vi, ti = wi.x * vi + wi.y * vr;  // w_i V
                const float2 o = make_float2(tr * wj.x + ti * wj.y, ti * wj.x - tr * wj.y);  // * conj(w_j)
                out = make_int2(__float_as_int(o.x), __float_as_int(o.y));
            }
            if (stage) stage[(ia - stage_r0) * VIS_LDS_STRIDE + (b - stage_c0)] = out;
            else vc[(size_t)ia * (ia + 1) / 2 + b] = out;
        }
        if (bs.mask) {
            // quad_perm [3, 3, 3, 3]: every lane of the quad reads lane 3's visibility
            const int yre = __builtin_amdgcn_mov_dpp(re, 0xFF, 0xF, 0xF, true);
            const int yim = __builtin_amdgcn_mov_dpp(im, 0xFF, 0xF, 0xF, true);
            const int bit = (2 * qq + h) * 8 + (cl >> 2);
            if ((lane & 3) == 0 && ((bs.mask >> bit) & 1ull)) {
                const int k = bs.base + __popcll(bs.mask & ((1ull << bit) - 1ull));
                // (V_XX + V_YY) / 2 rounded once to float.  |V| <= 2^15 n_spec, so for
                // n_spec <= 256 the sum is an integer below 2^24 and float arithmetic is exact
                // up to that one rounding (none), as the double form is.
                float2 v;
                if (small_sums) {
                    v = make_float2(0.5f * ((float)re + (float)yre), 0.5f * ((float)im + (float)yim));
                } else {
                    v = make_float2((float)(0.5 * ((double)re + (double)yre)), (float)(0.5 * ((double)im + (double)yim)));
                }
                so.out[(size_t)c * so.n_pairs + k] = v;
            }
        }
    }
}

// One 128 x 128 tile pair (I, J) of channel c: K loop through LDS, MFMA, epilogue.
// One TILE_I8 x TILE_I8 tile pair (I, J) of channel c; each of the four waves owns a WT x WT
// quarter (MI x MI MFMA tiles).  The K loop runs over KC-byte stages double buffered in LDS: the
// next stage's global loads are issued into registers before the current stage's MFMAs and
// stored to the other buffer after them, so one barrier per stage separates a buffer's last reads
// from its next writes.  LDS per workgroup: 2 stages x 2 operands x TILE_I8 x LDS_STRIDE bytes
// (40 KB), registers for four workgroups per CU.  Measured alternatives, slower on 704 inputs:
// 256 x 256 tiles with 128 x 128 per wave (one wave per SIMD: its LDS-to-MFMA and barrier waits
// are exposed), and register prefetch two stages ahead.
constexpr int TILE_LDS = TILE_I8 * LDS_STRIDE;
constexpr int WT = TILE_I8 / 2;  // a wave's share of the tile
constexpr int MI = WT / 32;      // MFMA tiles per wave per dimension
template <bool VEC, bool STOKES, bool CAL>
__device__ __forceinline__ void correlate_tile(const int8_t *__restrict__ q, int n_in, int T, int ldy, int c,
                                               int pair, int32_t *__restrict__ vis, int8_t *lds,
                                               const StokesOut &so, const float2 *__restrict__ calw,
                                               float2 *s_cal) {
    int I, J;
    tile_pair(pair, I, J);
    const int rows = 2 * n_in;
    const int8_t *Y = q + (size_t)c * rows * ldy;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int wr = wave >> 1, wc = wave & 1;
    const bool diag = (I == J);
    const bool active = !(diag && wr < wc);
    // stage buffers by offset (a runtime-indexed table of pointers would make every access a
    // generic flat instruction, which waits on the global loads in flight)
    auto sA = [lds](int bi) { return lds + 2 * bi * TILE_LDS; };
    auto sB = [lds](int bi) { return lds + (2 * bi + 1) * TILE_LDS; };

    v16i acc[MI][MI];
#pragma unroll
    for (int mi = 0; mi < MI; mi++)
#pragma unroll
        for (int ni = 0; ni < MI; ni++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[mi][ni][r] = 0;

    if (CAL) {  // correction factors of the tile's row and column inputs (WT / 2 each)
        const int in0 = I * (TILE_I8 / 2), jn0 = J * (TILE_I8 / 2);
        if (t < TILE_I8 / 2) s_cal[t] = in0 + t < n_in ? calw[(size_t)c * n_in + in0 + t] : make_float2(0.f, 0.f);
        else if (t < TILE_I8) {
            const int u = t - TILE_I8 / 2;
            s_cal[t] = jn0 + u < n_in ? calw[(size_t)c * n_in + jn0 + u] : make_float2(0.f, 0.f);
        }
    }
    const int n_st = (T + KC - 1) / KC;
    v4i ra[STAGE_VECS], rb[STAGE_VECS];
    load_stage<VEC>(ra, Y, rows, T, ldy, I * TILE_I8, 0, t);
    if (!diag) load_stage<VEC>(rb, Y, rows, T, ldy, J * TILE_I8, 0, t);
    store_stage(sA(0), ra, t);
    if (!diag) store_stage(sB(0), rb, t);
    __syncthreads();
    for (int st = 0; st < n_st; st++) {
        const int cur = st & 1;
        const bool more = st + 1 < n_st;
        if (more) {
            load_stage<VEC>(ra, Y, rows, T, ldy, I * TILE_I8, (st + 1) * KC, t);
            if (!diag) load_stage<VEC>(rb, Y, rows, T, ldy, J * TILE_I8, (st + 1) * KC, t);
        }
        if (active) {
            const int8_t *a_s = sA(cur) + (wr * WT + (lane & 31)) * LDS_STRIDE;
            const int8_t *b_s = (diag ? sA(cur) : sB(cur)) + (wc * WT + (lane & 31)) * LDS_STRIDE;
#pragma unroll
            for (int kk = 0; kk < KC; kk += 32) {
                const int koff = kk + (lane >> 5) * 16;
                v4i a[MI], b[MI];
#pragma unroll
                for (int mi = 0; mi < MI; mi++) a[mi] = *reinterpret_cast<const v4i *>(a_s + mi * 32 * LDS_STRIDE + koff);
#pragma unroll
                for (int ni = 0; ni < MI; ni++) b[ni] = *reinterpret_cast<const v4i *>(b_s + ni * 32 * LDS_STRIDE + koff);
#pragma unroll
                for (int mi = 0; mi < MI; mi++)
#pragma unroll
                    for (int ni = 0; ni < MI; ni++)
                        acc[mi][ni] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
            }
        }
        if (more) {
            store_stage(sA(cur ^ 1), ra, t);
            if (!diag) store_stage(sB(cur ^ 1), rb, t);
        }
        __syncthreads();
    }
    if (!active) return;
    const size_t nprod = (size_t)n_in * (n_in + 1) / 2;
    int2 *vc = reinterpret_cast<int2 *>(vis) + (size_t)c * nprod;
#pragma unroll
    for (int mi = 0; mi < MI; mi++)
#pragma unroll
        for (int ni = 0; ni < MI; ni++) {
            const int R0 = I * TILE_I8 + wr * WT + mi * 32;
            const int C0 = J * TILE_I8 + wc * WT + ni * 32;
            if (R0 < rows && C0 <= R0 + 31) {
                const BlockStokes bs = STOKES ? block_stokes(so, R0, C0) : BlockStokes();
                CalIn ci;
                if (CAL) ci = CalIn{s_cal, I * (TILE_I8 / 2), s_cal + TILE_I8 / 2, J * (TILE_I8 / 2)};
                store_tile_i32(acc[mi][ni], R0, C0, lane, n_in, vc, STOKES ? so : StokesOut(), c, bs, T <= 256, ci);
            }
        }
}

template <bool VEC, bool STOKES, bool CAL>
__global__ __launch_bounds__(256, 3) void correlate_i8_kernel(const int8_t *__restrict__ q, int n_chan,
                                                              int n_in, int T, int ldy, int n_pairs,
                                                              int32_t *__restrict__ vis, StokesOut so,
                                                              const float2 *__restrict__ calw) {
    __shared__ __attribute__((aligned(16))) int8_t lds[4 * TILE_LDS];
    __shared__ float2 s_cal[CAL ? TILE_I8 : 1];
    const int id = blockIdx.x;
    const int xcd = id & 7, rest = id >> 3;
    const int pair = rest % n_pairs;
    const int c = (rest / n_pairs) * 8 + xcd;
    if (c >= n_chan) return;
    correlate_tile<VEC, STOKES, CAL>(q, n_in, T, ldy, c, pair, vis, lds, so, calw, s_cal);
}

// Pipelined, persistent form of the tiled kernel for rows of a 16-byte multiple stride (every
// single-band launch; other integrations are repacked first), on PT x PT tiles of G (PT = 128:
// four waves, PT = 256: sixteen waves; each wave 64 x 64 of G).  A workgroup takes the tiles
// blockIdx.x, blockIdx.x + gridDim.x, ... (gridDim.x a multiple of 8, so every tile of a
// workgroup stays on its XCD) and runs their K stages as one stream: stage g of the workgroup is
// stage g mod n_st of its tile g / n_st.  A stage holds SK bytes of K of every row (64 for
// PT = 128, 128 for PT = 256: whole 128-byte lines of L2, read once) and the stages go through a
// ring of DEPTH LDS buffers (3 x 48 KB for PT = 128, 2 x 64 KB for PT = 256) filled by
// direct-to-LDS buffer loads (no registers, no LDS store instructions): while stage g is
// multiplied the loads of the next DEPTH - 1 stages are in flight, also across the end of a tile,
// so a tile's first loads run under the previous tile's epilogue (with 128 KB of LDS one
// workgroup holds a CU).  A wave's load writes 1 KB of LDS (1024 / SK rows); row r keeps its
// 16-byte K chunks in the order slot(j, r), so the fragment reads of 16 consecutive rows at one
// chunk hit distinct banks.  Reads past the channel's rows or past the row stride go beyond the
// buffer's range and return 0.  Waits are explicit: each thread waits for its own loads of stage
// g (later stages may stay outstanding), then a barrier makes every thread's loads visible and
// frees the buffer that the next loads overwrite (read one stage earlier).  Within a stage the
// fragments of the next 32-byte K block are read while the current block multiplies.  Long
// integrations take the 256 x 256 tile, which moves half the operand bytes from L2 per
// multiply-add.  (Measured at 704 inputs, T = 2,048: neither the barriers nor the waits cost
// time; eight waves of 128 x 64 are slower than sixteen of 64 x 64; the clock under this load
// settles near 1.9 GHz.)
typedef __attribute__((address_space(3))) void lds_void_t;

template <int PT>
struct PipeShape {
    static constexpr int SK = PT == 128 ? 64 : 128;   // bytes of K per stage and row
    static constexpr int DEPTH = PT == 128 ? 3 : 2;   // stages in the LDS ring
    static constexpr int WPB = PT == 128 ? 3 : 1;     // workgroups per CU
    static constexpr int WM = 64;                     // rows of G per wave
    static constexpr int WN = 64;                     // columns of G per wave
    static constexpr int MI = WM / 32, NI = WN / 32;  // 32 x 32 MFMA blocks per wave
    static constexpr int WR = PT / WM, WC = PT / WN;  // wave grid WR x WC
    static constexpr int NW = WR * WC;                // waves
    static constexpr int CPR = SK / 16;               // 16-byte chunks per row
    static constexpr int RPK = 1024 / SK;             // rows per 1 KB block
    static constexpr int OP = PT * SK;                // bytes of one operand's stage
    static constexpr int STAGE = 2 * OP;              // bytes of a stage
    static constexpr int BPW = PT / RPK / NW;         // 1 KB blocks per operand and wave
    static constexpr int LOADS = 2 * BPW;             // direct loads per thread and stage
    static_assert(BPW >= 1 && (PT / RPK) % NW == 0, "whole blocks per wave");
    // slot of chunk j in row r: rows r .. r + 255 / SK share the 256 bytes of the 64 banks, and
    // 16 consecutive rows read at one chunk hit 16 distinct 16-byte bank groups
    static __device__ __forceinline__ int slot(int j, int r) { return j ^ ((r / (256 / SK)) & (CPR - 1)); }
};

template <int N>
__device__ __forceinline__ void wait_vm() {  // s_waitcnt vmcnt(N), other counters untouched
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Wait until at most `stages` stages of this thread's loads (LOADS each) are outstanding.
template <int LOADS, int MAXST>
__device__ __forceinline__ void wait_stages(int stages) {
    if (MAXST >= 2 && stages >= 2) wait_vm<2 * LOADS>();
    else if (stages >= 1) wait_vm<LOADS>();
    else wait_vm<0>();
}

__device__ __forceinline__ void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Tile u of workgroup b: tile id b + u gridDim.x -> XCD lane id & 7, pair, channel.
struct PipeTile {
    int c, I, J;
};

__device__ __forceinline__ PipeTile pipe_tile(int rest, int xcd, int n_pairs) {
    PipeTile p;
    p.c = (rest / n_pairs) * 8 + xcd;
    tile_pair(rest % n_pairs, p.I, p.J);
    return p;
}

template <int PT, bool STOKES, bool CAL>
__global__ __launch_bounds__(64 * PipeShape<PT>::NW, PipeShape<PT>::WPB) void correlate_i8_pipe_kernel(
    const int8_t *__restrict__ q, int n_chan, int n_in, int T, int ldy, int n_pairs, int32_t *__restrict__ vis,
    StokesOut so, const float2 *__restrict__ calw) {
    using PS = PipeShape<PT>;
    __shared__ __attribute__((aligned(16))) int8_t lds[PS::DEPTH * PS::STAGE];
    __shared__ float2 s_cal[CAL ? PT : 1];
    const int rows = 2 * n_in;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    // this workgroup's tiles: rest = rest0 + u step for u = 0 .. n_tiles - 1 (the channels of the
    // last group of eight that do not exist end the list of the XCD lanes past them)
    const int xcd = blockIdx.x & 7, rest0 = blockIdx.x >> 3, step = gridDim.x >> 3;
    const int n_groups = (n_chan + 7) / 8;
    const int rest_end = (xcd < n_chan - 8 * (n_groups - 1) ? n_groups : n_groups - 1) * n_pairs;
    const int n_tiles = rest0 < rest_end ? (rest_end - 1 - rest0) / step + 1 : 0;
    const int n_st = (T + PS::SK - 1) / PS::SK;
    const int n_g = n_tiles * n_st;
    if (n_g == 0) return;

    // this thread's loads: wave w fills 1 KB blocks BPW w .. BPW w + BPW - 1 of each operand
    // (rows 16 b .. 16 b + 15: the lane's row l / 4 and slot l % 4 of the block)
    int rl[PS::BPW], slot_chunk[PS::BPW];
#pragma unroll
    for (int i = 0; i < PS::BPW; i++) {
        rl[i] = (PS::BPW * wave + i) * PS::RPK + lane / PS::CPR;
        slot_chunk[i] = PS::slot(lane % PS::CPR, rl[i]);  // the K chunk this lane's slot holds (an involution)
    }
    // loads of stream stage g: tile ti (stage s of it) into ring buffer g mod DEPTH
    PipeTile li = pipe_tile(rest0, xcd, n_pairs);
    int l_tile = 0, l_s = 0;
    auto issue_next = [&](int g) __attribute__((always_inline)) {
        const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<int8_t *>(q + (size_t)li.c * rows * ldy), (short)0, rows * ldy, 0x00020000);
        int8_t *base = lds + (g % PS::DEPTH) * PS::STAGE;
        const bool ldiag = li.I == li.J;
#pragma unroll
        for (int i = 0; i < PS::BPW; i++) {
            const int k = l_s * PS::SK + 16 * slot_chunk[i];
            const int ra = li.I * PT + rl[i];
            const int rb = ldiag ? rows : li.J * PT + rl[i];  // (diagonal tiles read A only)
            const unsigned va = (ra < rows && k < ldy) ? (unsigned)(ra * ldy + k) : 0x80000000u;
            const unsigned vb = (rb < rows && k < ldy) ? (unsigned)(rb * ldy + k) : 0x80000000u;
            int8_t *blk = base + (PS::BPW * wave + i) * 1024;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_void_t *)blk, 16, va, 0, 0, 0);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_void_t *)(blk + PS::OP), 16, vb, 0, 0, 0);
        }
        if (++l_s == n_st) {
            l_s = 0;
            if (++l_tile < n_tiles) li = pipe_tile(rest0 + l_tile * step, xcd, n_pairs);
        }
    };

    v16i acc[PS::MI][PS::NI];
#pragma unroll
    for (int mi = 0; mi < PS::MI; mi++)
#pragma unroll
        for (int ni = 0; ni < PS::NI; ni++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[mi][ni][r] = 0;
#pragma unroll
    for (int g = 0; g < PS::DEPTH - 1; g++)
        if (g < n_g) issue_next(g);

    const size_t nprod = (size_t)n_in * (n_in + 1) / 2;
    PipeTile ct = pipe_tile(rest0, xcd, n_pairs);
    int c_tile = 0, s = 0;
    for (int g = 0; g < n_g; g++) {
        const bool diag = ct.I == ct.J;
        // the wave's block of the tile (wr, wc); on a diagonal tile of sixteen waves the ten
        // blocks on or below the diagonal are spread 3, 3, 2, 2 over the SIMDs (wave w runs on
        // SIMD w mod 4) instead of 4, 3, 2, 1
        const int pos = (PS::NW == 16 && diag) ? (int)((0xB62173A5FD94EC80ull >> (4 * wave)) & 15) : wave;
        const int wr = pos / PS::WC, wc = pos % PS::WC;
        // fragment rows of this wave (A: wr, B: wc); a row's chunk j sits at slot(j, r)
        const int ra0 = wr * PS::WM + (lane & 31), rb0 = wc * PS::WN + (lane & 31);
        // waves wholly above the diagonal of a diagonal tile, or wholly past the last row, multiply nothing
        const bool active = !(diag && wc * PS::WN > wr * PS::WM + PS::WM - 1) && ct.I * PT + wr * PS::WM < rows;
        // stages g + 1 .. g + DEPTH - 2 may stay in flight
        wait_stages<PS::LOADS, PS::DEPTH - 2>(min(n_g - 1 - g, PS::DEPTH - 2));
        lds_barrier();
        if (g + PS::DEPTH - 1 < n_g) issue_next(g + PS::DEPTH - 1);
        if (CAL && s == 0) {  // correction factors of the tile's row and column inputs (PT / 2 each)
            for (int u = t; u < PT; u += 64 * PS::NW) {
                const int in = u < PT / 2 ? ct.I * (PT / 2) + u : ct.J * (PT / 2) + u - PT / 2;
                s_cal[u] = in < n_in ? calw[(size_t)ct.c * n_in + in] : make_float2(0.f, 0.f);
            }
        }
        if (active) {
            const int8_t *sa = lds + (g % PS::DEPTH) * PS::STAGE;
            const int8_t *sb = diag ? sa : sa + PS::OP;
            // fragments of K block kk (32 bytes: the lane's half j = 2 kk + l / 32)
            auto frag = [&](int kk, v4i *a, v4i *b) __attribute__((always_inline)) {
                const int j = 2 * kk + (lane >> 5);
#pragma unroll
                for (int mi = 0; mi < PS::MI; mi++) {
                    const int r = ra0 + mi * 32;
                    a[mi] = *reinterpret_cast<const v4i *>(sa + r * PS::SK + (PS::slot(j, r) << 4));
                }
#pragma unroll
                for (int ni = 0; ni < PS::NI; ni++) {
                    const int r = rb0 + ni * 32;
                    b[ni] = *reinterpret_cast<const v4i *>(sb + r * PS::SK + (PS::slot(j, r) << 4));
                }
            };
            auto mma = [&](const v4i *a, const v4i *b) __attribute__((always_inline)) {
#pragma unroll
                for (int mi = 0; mi < PS::MI; mi++)
#pragma unroll
                    for (int ni = 0; ni < PS::NI; ni++)
                        acc[mi][ni] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
            };
            constexpr int NK = PS::SK / 32;
            // the fragments of block kk + 1 load while block kk multiplies (blocks past T hold 0)
            // (scheduling barriers keep the compiler from pulling the reads back behind the MFMAs)
            v4i a[2][PS::MI], b[2][PS::NI];
            frag(0, a[0], b[0]);
#pragma unroll
            for (int kk = 0; kk < NK; kk++) {
                if (kk + 1 < NK) frag(kk + 1, a[(kk + 1) & 1], b[(kk + 1) & 1]);
                __builtin_amdgcn_sched_barrier(0);
                mma(a[kk & 1], b[kk & 1]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        if (++s < n_st) continue;
        // the tile's last stage: epilogue (the next tile's first stages are already loading)
        if (CAL) lds_barrier();  // s_cal visible to every wave
        if (active) {
            int2 *vc = reinterpret_cast<int2 *>(vis) + (size_t)ct.c * nprod;
#pragma unroll
            for (int mi = 0; mi < PS::MI; mi++)
#pragma unroll
                for (int ni = 0; ni < PS::NI; ni++) {
                    const int R0 = ct.I * PT + wr * PS::WM + mi * 32;
                    const int C0 = ct.J * PT + wc * PS::WN + ni * 32;
                    if (R0 < rows && C0 <= R0 + 31) {
                        const BlockStokes bs = STOKES ? block_stokes(so, R0, C0) : BlockStokes();
                        CalIn ci;
                        if (CAL) ci = CalIn{s_cal, ct.I * (PT / 2), s_cal + PT / 2, ct.J * (PT / 2)};
                        store_tile_i32(acc[mi][ni], R0, C0, lane, n_in, vc, STOKES ? so : StokesOut(), ct.c, bs,
                                       T <= 256, ci);
                    }
                }
        }
#pragma unroll
        for (int mi = 0; mi < PS::MI; mi++)
#pragma unroll
            for (int ni = 0; ni < PS::NI; ni++)
#pragma unroll
                for (int r = 0; r < 16; r++) acc[mi][ni][r] = 0;
        s = 0;
        if (++c_tile < n_tiles) ct = pipe_tile(rest0 + c_tile * step, xcd, n_pairs);
    }
}

// Several sub-bands in one launch: task -> (job, channel group of 8, tile pair, XCD lane), one
// workgroup per task, in the same XCD-preserving order as the single-band launch.
template <bool VEC>
__global__ __launch_bounds__(256, 3) void correlate_i8_batch_kernel(const CorrJob *__restrict__ jobs, int n_jobs,
                                                                    int n_tasks) {
    __shared__ __attribute__((aligned(16))) int8_t lds[4 * TILE_LDS];
    const int task = blockIdx.x;
    if (task >= n_tasks) return;
    int j = 0;
    while (j + 1 < n_jobs && jobs[j + 1].task0 <= task) j++;
    const CorrJob jb = jobs[j];
    const int local = task - jb.task0;
    const int n_tiles = (2 * jb.n_in + TILE_I8 - 1) / TILE_I8;
    const int n_pairs = n_tiles * (n_tiles + 1) / 2;
    const int xcd = local & 7, rest = local >> 3;
    const int pair = rest % n_pairs;
    const int c = (rest / n_pairs) * 8 + xcd;
    if (c < jb.n_chan)
        correlate_tile<VEC, false, false>(jb.q, jb.n_in, jb.n_spec, jb.n_spec, c, pair, jb.vis, lds, StokesOut(),
                                          nullptr, nullptr);
}

// Repack int8 rows of T bytes to a stride of ldy bytes (ldy >= T, a multiple of 16), zero-filled,
// so the tiled correlator stages whole 16-byte vectors.  One thread per 16-byte output vector.
// Repack rows of T bytes to a stride of ldy (a multiple of 16 above T), zero-filled.  One thread
// per 16-byte output chunk reads the five aligned words around its 16 bytes (the source is
// 16-byte aligned, so a row starts at any byte of a word) and shifts them into place with
// v_alignbyte; a row's last, partial chunk is read byte by byte.
__global__ __launch_bounds__(256) void pad_rows_kernel(const int8_t *__restrict__ src, size_t n_rows, int T,
                                                       int ldy, int8_t *__restrict__ dst) {
    const size_t vpr = (size_t)(ldy / 16);
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n_rows * vpr) return;
    const size_t r = e / vpr;
    const int k = (int)(e % vpr) * 16;
    const size_t a = r * (size_t)T + k;  // first source byte
    v4i out;
    if (k + 16 <= T && (a & ~(size_t)3) + 20 <= n_rows * (size_t)T) {
        const uint32_t *w = reinterpret_cast<const uint32_t *>(src + (a & ~(size_t)3));
        const unsigned sh = (unsigned)(a & 3);
        uint32_t x[5];
#pragma unroll
        for (int i = 0; i < 5; i++) x[i] = w[i];
#pragma unroll
        for (int i = 0; i < 4; i++) out[i] = (int)__builtin_amdgcn_alignbyte(x[i + 1], x[i], sh);
    } else {
        int8_t tmp[16];
        const int8_t *s = src + a;
#pragma unroll
        for (int b = 0; b < 16; b++) tmp[b] = (k + b < T) ? s[b] : (int8_t)0;
        out = *reinterpret_cast<v4i *>(tmp);
    }
    *reinterpret_cast<v4i *>(dst + r * (size_t)ldy + k) = out;
}

// Short integrations (n_spec <= 64): one workgroup per channel keeps the channel's whole
// int8 matrix Y (2 n_in rows x n_spec, zero-padded to 32 or 64) in LDS and each wave walks a
// 32-row panel of G across every column tile at or left of the diagonal, so the packed
// triangle rows of its 16 inputs are written as consecutive 128-byte segments by one wave
// (whole cache lines form in L2 promptly).  At these sizes the write of the visibilities is
// the bound, not the matrix cores.  (Measured: 8 waves per workgroup, or panels handed out
// largest first, write more slowly; nontemporal stores, which skip the merging of the partial
// lines at segment edges in L2, 2.4x more slowly; staging four or two tiles' rows in LDS so each
// store writes one row segment of 64 or 32 products, 3% and 5% more slowly.  A store-only probe
// of this pattern takes as long as the kernel; writing each triangle row whole before the next
// takes 40% less there, but a wave's 16 rows advance together across its panel, and a kernel
// that stages a whole panel's rows in LDS to write them row by row fits one workgroup per CU
// and ran 1.4x more slowly.)
// The grid is CHAN_GRID workgroups (1.5 per CU of the 256-CU part) that walk the channels in
// strides of the grid: fewer writers in flight per L2 than one workgroup per channel, and the
// launch of 4,096 channels at 704 inputs writes 14% faster (384 was the fastest of grids from
// 288 to 512; 256 or fewer leave the write path idle while a channel is staged).
constexpr int CHAN_WAVES = 4;
constexpr int CHAN_GRID = 384;
template <int KP>  // padded K: 32 or 64
__device__ __forceinline__ void correlate_channel(const int8_t *__restrict__ q, int n_in, int T, int c,
                                                  int32_t *__restrict__ vis, int8_t *sY, const StokesOut &so,
                                                  const float2 *__restrict__ calw) {
    constexpr int NT = 64 * CHAN_WAVES;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int rows = 2 * n_in;
    const int n_panels = (rows + 31) / 32;
    const int rows_pad = n_panels * 32;
    const int8_t *Y = q + (size_t)c * rows * T;
    // stage Y: 16-byte vectors when rows are whole vectors, else bytes, zero-padded
    if (T == KP) {
        const v4i *src = reinterpret_cast<const v4i *>(Y);
        v4i *dst = reinterpret_cast<v4i *>(sY);
        const int nv = rows * KP / 16;
        for (int e = t; e < nv; e += NT) dst[e] = src[e];
        for (int e = nv + t; e < rows_pad * KP / 16; e += NT) dst[e] = v4i{0, 0, 0, 0};
    } else {
        for (int e = t; e < rows_pad * KP; e += NT) {
            const int r = e / KP, k = e % KP;
            sY[e] = (r < rows && k < T) ? Y[(size_t)r * T + k] : (int8_t)0;
        }
    }
    CalIn ci;
    if (calw) {  // channel c's correction factors, after Y in dynamic LDS
        float2 *sw = reinterpret_cast<float2 *>(sY + rows_pad * KP);
        for (int e = t; e < n_in; e += NT) sw[e] = calw[(size_t)c * n_in + e];
        ci = CalIn{sw, 0, sw, 0};
    }
    __syncthreads();
    const size_t nprod = (size_t)n_in * (n_in + 1) / 2;
    int2 *vc = reinterpret_cast<int2 *>(vis) + (size_t)c * nprod;
    const int koff = (lane >> 5) * 16;
    const int rl = lane & 31;
    // panel I (32 rows of G, 16 inputs) goes to wave I % 4, reversed on every other block of
    // four, so the waves get similar numbers of tiles (panel I has I + 1 of them)
    static_assert(CHAN_WAVES == 4, "panel assignment for four waves");
    for (int I = 0; I < n_panels; I++) {
        const int pos = I & 3;
        if ((((I >> 2) & 1) ? 3 - pos : pos) != wave) continue;
        v4i a[KP / 32];
#pragma unroll
        for (int kk = 0; kk < KP / 32; kk++)
            a[kk] = *reinterpret_cast<const v4i *>(sY + (I * 32 + rl) * KP + kk * 32 + koff);
        for (int J = 0; J <= I; J++) {
            const BlockStokes bs = block_stokes(so, I * 32, J * 32);  // issued before the MFMA
            v16i acc;
#pragma unroll
            for (int r = 0; r < 16; r++) acc[r] = 0;
#pragma unroll
            for (int kk = 0; kk < KP / 32; kk++) {
                const v4i b = *reinterpret_cast<const v4i *>(sY + (J * 32 + rl) * KP + kk * 32 + koff);
                acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[kk], b, acc, 0, 0, 0);
            }
            store_tile_i32(acc, I * 32, J * 32, lane, n_in, vc, so, c, bs, true, ci);  // n_spec <= KP <= 64
        }
    }
}

template <int KP>
__global__ __launch_bounds__(64 * CHAN_WAVES) void correlate_i8_chan_kernel(const int8_t *__restrict__ q, int n_chan,
                                                                            int n_in, int T,
                                                                            int32_t *__restrict__ vis, StokesOut so,
                                                                            const float2 *__restrict__ calw) {
    extern __shared__ __attribute__((aligned(16))) int8_t sY[];  // [rows_pad][KP], then [n_in] float2 with calw
    for (int c = blockIdx.x; c < n_chan; c += gridDim.x) {
        if (c != (int)blockIdx.x) __syncthreads();  // every wave is done with the previous channel's LDS
        correlate_channel<KP>(q, n_in, T, c, vis, sY, so, calw);
    }
}

template <int KP>
__global__ __launch_bounds__(64 * CHAN_WAVES) void correlate_i8_chan_batch_kernel(const CorrJob *__restrict__ jobs,
                                                                                  int n_jobs, int n_tasks) {
    extern __shared__ __attribute__((aligned(16))) int8_t sY[];
    const int task = blockIdx.x;  // one workgroup per channel of any job
    if (task >= n_tasks) return;
    int j = 0;
    while (j + 1 < n_jobs && jobs[j + 1].task0 <= task) j++;
    const CorrJob jb = jobs[j];
    correlate_channel<KP>(jb.q, jb.n_in, jb.n_spec, task - jb.task0, jb.vis, sY, StokesOut(), nullptr);
}

// ---- plain FP32 path: the same Gram formulation on v_mfma_f32_32x32x2_f32 ----
typedef float v16f __attribute__((ext_vector_type(16)));
constexpr int KCF = 16;  // K floats per LDS stage
constexpr int LDS_STRIDE_F = KCF + 1;

__device__ __forceinline__ float swap_lanes_f(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, true));
}

__global__ __launch_bounds__(256) void correlate_f32_kernel(const float *__restrict__ q, int n_chan,
                                                            int n_in, int T, int n_pairs,
                                                            float *__restrict__ vis) {
    __shared__ float sA[TILE * LDS_STRIDE_F];
    __shared__ float sB[TILE * LDS_STRIDE_F];
    const int id = blockIdx.x;
    const int xcd = id & 7, rest = id >> 3;
    const int pair = rest % n_pairs;
    const int c = (rest / n_pairs) * 8 + xcd;
    if (c >= n_chan) return;
    int I, J;
    tile_pair(pair, I, J);
    const int rows = 2 * n_in;
    const float *Y = q + (size_t)c * rows * T;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int wr = wave >> 1, wc = wave & 1;
    const bool diag = (I == J);
    const bool active = !(diag && wr < wc);
    v16f acc[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; mi++)
#pragma unroll
        for (int ni = 0; ni < 2; ni++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[mi][ni][r] = 0.f;
    const float *sBr = diag ? sA : sB;
    for (int k0 = 0; k0 < T; k0 += KCF) {
        __syncthreads();
        for (int e = t; e < TILE * KCF; e += 256) {
            const int rl = e / KCF, kk = e % KCF;
            const int r = I * TILE + rl, k = k0 + kk;
            sA[rl * LDS_STRIDE_F + kk] = (r < rows && k < T) ? Y[(size_t)r * T + k] : 0.f;
            if (!diag) {
                const int r2 = J * TILE + rl;
                sB[rl * LDS_STRIDE_F + kk] = (r2 < rows && k < T) ? Y[(size_t)r2 * T + k] : 0.f;
            }
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int kk = 0; kk < KCF; kk += 2) {
                const int koff = kk + (lane >> 5);
                float a[2], b[2];
#pragma unroll
                for (int mi = 0; mi < 2; mi++) a[mi] = sA[(wr * 64 + mi * 32 + (lane & 31)) * LDS_STRIDE_F + koff];
#pragma unroll
                for (int ni = 0; ni < 2; ni++) b[ni] = sBr[(wc * 64 + ni * 32 + (lane & 31)) * LDS_STRIDE_F + koff];
#pragma unroll
                for (int mi = 0; mi < 2; mi++)
#pragma unroll
                    for (int ni = 0; ni < 2; ni++)
                        acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
            }
        }
    }
    if (!active) return;
    const size_t nprod = (size_t)n_in * (n_in + 1) / 2;
    float2 *vc = reinterpret_cast<float2 *>(vis) + (size_t)c * nprod;
    const int p = lane & 1, h = lane >> 5, cl = lane & 31;
#pragma unroll
    for (int mi = 0; mi < 2; mi++)
#pragma unroll
        for (int ni = 0; ni < 2; ni++) {
            const int R0 = I * TILE + wr * 64 + mi * 32;
            const int C0 = J * TILE + wc * 64 + ni * 32;
            if (!(R0 < rows && C0 <= R0 + 31)) continue;
            const v16f &a = acc[mi][ni];
            float par[16];
#pragma unroll
            for (int r = 0; r < 16; r++) par[r] = swap_lanes_f(a[r]);
            const int b = (C0 >> 1) + (cl >> 1);
#pragma unroll
            for (int qq = 0; qq < 4; qq++) {
                const int ia = (R0 >> 1) + 4 * qq + 2 * h + p;
                float re, im;
                if (p == 0) {
                    re = a[4 * qq] + par[4 * qq + 1];
                    im = a[4 * qq + 1] - par[4 * qq];
                } else {
                    re = par[4 * qq + 2] + a[4 * qq + 3];
                    im = par[4 * qq + 3] - a[4 * qq + 2];
                }
                if (ia < n_in && b <= ia) vc[(size_t)ia * (ia + 1) / 2 + b] = make_float2(re, im);
            }
        }
}

}  // namespace

hipError_t launch_correlate_i8(const int8_t *q, int n_chan, int n_in, int n_spec, int32_t *vis,
                               hipStream_t st, StokesOut so, int8_t *pad_scratch, const float2 *calw) {
    return launch_correlate_variant(q, n_chan, n_in, n_spec, vis, correlate_default_variant(n_in, n_spec), st, so,
                                    pad_scratch, calw);
}

size_t correlate_pad_bytes(int n_chan, int n_in, int n_spec) {
    if (correlate_default_variant(n_in, n_spec) != CORR_VARIANT_TILED || (n_spec & 15) == 0) return 0;
    return (size_t)n_chan * 2 * n_in * (size_t)((n_spec + 15) & ~15);
}

size_t correlate_chan_lds(int n_in, int variant) {
    const int kp = variant == CORR_VARIANT_CHAN64 ? 64 : 32;
    return (size_t)((2 * n_in + 31) / 32) * 32 * kp;
}

// Tasks of a batched correlator launch for one job and variant.
int correlate_batch_tasks(const CorrJob &jb, int variant) {
    if (variant == CORR_VARIANT_TILED) {
        const int n_tiles = (2 * jb.n_in + TILE_I8 - 1) / TILE_I8;
        return ((jb.n_chan + 7) / 8) * 8 * (n_tiles * (n_tiles + 1) / 2);
    }
    return jb.n_chan;
}

// The whole-channel kernels hold the channel's matrix in LDS (at most CHAN_LDS_MAX bytes); they
// serve short integrations.
constexpr int CHAN_LDS_MAX = 96 * 1024;

bool correlate_variant_valid(int n_in, int n_spec, int variant) {
    if (variant == CORR_VARIANT_TILED) return true;
    if (variant == CORR_VARIANT_CHAN32) return n_spec <= 32 && correlate_chan_lds(n_in, variant) <= (size_t)CHAN_LDS_MAX;
    if (variant == CORR_VARIANT_CHAN64) return n_spec <= 64 && correlate_chan_lds(n_in, variant) <= (size_t)CHAN_LDS_MAX;
    return false;
}

int correlate_default_variant(int n_in, int n_spec) {
    if (correlate_variant_valid(n_in, n_spec, CORR_VARIANT_CHAN32)) return CORR_VARIANT_CHAN32;
    if (correlate_variant_valid(n_in, n_spec, CORR_VARIANT_CHAN64)) return CORR_VARIANT_CHAN64;
    return CORR_VARIANT_TILED;
}

// The whole-channel kernels can need more than the default 64 KB of dynamic LDS: raise the limit
// of all four to the largest size a valid shape uses, once per device (outside any capture).
hipError_t chan_lds_prepare() {
    static std::mutex mu;
    static std::vector<int> done;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (std::find(done.begin(), done.end(), dev) != done.end()) return hipSuccess;
    const void *fns[] = {(const void *)correlate_i8_chan_kernel<32>, (const void *)correlate_i8_chan_kernel<64>,
                         (const void *)correlate_i8_chan_batch_kernel<32>,
                         (const void *)correlate_i8_chan_batch_kernel<64>};
    for (const void *f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, CHAN_LDS_MAX);
        if (e != hipSuccess) return e;
    }
    done.push_back(dev);
    return hipSuccess;
}

hipError_t correlate_batch_prepare(int variant, int n_in) {
    (void)n_in;
    return variant == CORR_VARIANT_TILED ? hipSuccess : chan_lds_prepare();
}

hipError_t launch_correlate_batch(const CorrJob *d_jobs, int n_jobs, int n_tasks, int variant, int n_in, bool vec,
                                  hipStream_t st) {
    if (variant == CORR_VARIANT_TILED) {
        if (vec) hipLaunchKernelGGL(correlate_i8_batch_kernel<true>, dim3(n_tasks), dim3(256), 0, st, d_jobs, n_jobs, n_tasks);
        else hipLaunchKernelGGL(correlate_i8_batch_kernel<false>, dim3(n_tasks), dim3(256), 0, st, d_jobs, n_jobs, n_tasks);
        return hipGetLastError();
    }
    const size_t lds = correlate_chan_lds(n_in, variant);
    if (variant == CORR_VARIANT_CHAN32)
        hipLaunchKernelGGL(correlate_i8_chan_batch_kernel<32>, dim3(n_tasks), dim3(64 * CHAN_WAVES), lds, st, d_jobs,
                           n_jobs, n_tasks);
    else
        hipLaunchKernelGGL(correlate_i8_chan_batch_kernel<64>, dim3(n_tasks), dim3(64 * CHAN_WAVES), lds, st, d_jobs,
                           n_jobs, n_tasks);
    return hipGetLastError();
}

// Compute units of the current device (queried once per device).
static int device_cus() {
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        int n = 0;
        cus[dev] = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0 ? n : 256;
    }
    return cus[dev];
}

// Single-band launch of one variant (the default path and the autotuner's candidates).
hipError_t launch_correlate_variant(const int8_t *q, int n_chan, int n_in, int n_spec, int32_t *vis, int variant,
                                    hipStream_t st, StokesOut so, int8_t *pad_scratch, const float2 *calw) {
    // the whole-channel kernels keep the correction factors after Y in LDS; when that does not
    // fit the tiled kernel (which stages only its tile's factors) takes the channel
    if (calw && variant != CORR_VARIANT_TILED &&
        correlate_chan_lds(n_in, variant) + sizeof(float2) * n_in > (size_t)CHAN_LDS_MAX)
        variant = CORR_VARIANT_TILED;
    if (variant == CORR_VARIANT_TILED) {
        int ldy = n_spec;
        if ((n_spec & 15) && pad_scratch) {
            ldy = (n_spec + 15) & ~15;
            const size_t n_rows = (size_t)n_chan * 2 * n_in;
            const size_t n_vec = n_rows * (size_t)(ldy / 16);
            hipLaunchKernelGGL(pad_rows_kernel, dim3((unsigned)((n_vec + 255) / 256)), dim3(256), 0, st, q, n_rows,
                               n_spec, ldy, pad_scratch);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            q = pad_scratch;
        }
        const int n_tiles = (2 * n_in + TILE_I8 - 1) / TILE_I8;
        const int n_pairs = n_tiles * (n_tiles + 1) / 2;
        const size_t groups = (size_t)((n_chan + 7) / 8) * 8 * n_pairs;
#define NBSI_TILED(V, S, CL)                                                                                    \
    hipLaunchKernelGGL((correlate_i8_kernel<V, S, CL>), dim3((unsigned)groups), dim3(256), 0, st, q, n_chan, n_in, \
                       n_spec, ldy, n_pairs, vis, so, calw)
        if (ldy & 15) {
            if (calw) NBSI_TILED(false, false, true);
            else if (so.out) NBSI_TILED(false, true, false);
            else NBSI_TILED(false, false, false);
        } else {
            const int pt = n_spec >= PIPE_BIG_T ? 256 : 128;
            const int nt = (2 * n_in + pt - 1) / pt, np = nt * (nt + 1) / 2;
            // persistent grid: the resident workgroups, a multiple of 8, no more than the tiles
            const size_t tiles = (size_t)((n_chan + 7) / 8) * 8 * np;
            const size_t g = std::min(tiles, (size_t)device_cus() * (pt == 256 ? PipeShape<256>::WPB : PipeShape<128>::WPB) / 8 * 8);
#define NBSI_PIPE(PT, S, CL)                                                                                         \
    hipLaunchKernelGGL((correlate_i8_pipe_kernel<PT, S, CL>), dim3((unsigned)g), dim3(64 * PipeShape<PT>::NW), 0, st, q, \
                       n_chan, n_in, n_spec, ldy, np, vis, so, calw)
            if (pt == 256) {
                if (calw) NBSI_PIPE(256, false, true);
                else if (so.out) NBSI_PIPE(256, true, false);
                else NBSI_PIPE(256, false, false);
            } else {
                if (calw) NBSI_PIPE(128, false, true);
                else if (so.out) NBSI_PIPE(128, true, false);
                else NBSI_PIPE(128, false, false);
            }
#undef NBSI_PIPE
        }
#undef NBSI_TILED
        return hipGetLastError();
    }
    const size_t lds = correlate_chan_lds(n_in, variant) + (calw ? sizeof(float2) * n_in : 0);
    const hipError_t e = chan_lds_prepare();
    if (e != hipSuccess) return e;
    if (variant == CORR_VARIANT_CHAN32)
        hipLaunchKernelGGL(correlate_i8_chan_kernel<32>, dim3(std::min(n_chan, CHAN_GRID)), dim3(64 * CHAN_WAVES), lds, st, q, n_chan, n_in,
                           n_spec, vis, so, calw);
    else
        hipLaunchKernelGGL(correlate_i8_chan_kernel<64>, dim3(std::min(n_chan, CHAN_GRID)), dim3(64 * CHAN_WAVES), lds, st, q, n_chan, n_in,
                           n_spec, vis, so, calw);
    return hipGetLastError();
}

hipError_t launch_correlate_f32(const float *q, int n_chan, int n_in, int n_spec, float *vis,
                                hipStream_t st) {
    const int n_tiles = (2 * n_in + TILE - 1) / TILE;
    const int n_pairs = n_tiles * (n_tiles + 1) / 2;
    const size_t groups = (size_t)((n_chan + 7) / 8) * 8 * n_pairs;
    hipLaunchKernelGGL(correlate_f32_kernel, dim3((unsigned)groups), dim3(256), 0, st, q, n_chan, n_in,
                       n_spec, n_pairs, vis);
    return hipGetLastError();
}
