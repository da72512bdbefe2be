// Candidate classifier on FP16 matrix cores: stamp extraction, forward pass, backward pass and
// Adam, with FP32 master weights and FP32 accumulation.  The network stands in for the paper's
// Stage II screen of Stage I candidates (Sec. 2.4); its shape is this library's own choice:
// conv3x3(33 -> 32) - ReLU - conv3x3(32 -> 64) - ReLU - conv3x3(64 -> 32) - ReLU -
// global average pool - linear(32 -> 1), trained with binary cross-entropy on the logit.
//
// Every convolution is an implicit GEMM on gfx950's v_mfma_f32_32x32x16_f16 (K = 16 per
// instruction: lanes 0-31 carry k 0..7 of their row or column, lanes 32-63 k 8..15): rows are
// (stamp, position) pairs of the batch (81 positions per 9 x 9 stamp), columns output channels,
// and the reduction runs over (tap, input channel) with k = tap * CINP + ci (input channels
// padded to a multiple of 16 with zero weights).  Activations are stored position-major with
// the channel fastest, [b][81][C], so one lane's eight consecutive k are one 16-byte load.
//
// Backward: gradients leave the loss in FP32; before each FP16 product they are scaled by a
// power of two chosen from their maximum (the first from a bound, later ones from an exact
// maximum taken with an order-independent integer max), so the FP16 values use the top of the
// format's range; every weight gradient is divided by its scale in FP32 at the end.  Weight
// gradients are split over the batch into fixed partial sums reduced in a fixed order: the
// results are deterministic.
#include "internal.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

namespace {

typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int SC = NBSI_STAMP_CHANNELS;   // 33 spectral channels per stamp
constexpr int SP = NBSI_STAMP_PIXELS;     // 9 x 9 pixels
constexpr int NPOS = SP * SP;
constexpr int HALF_C = SC / 2, HALF_P = SP / 2;

// flat parameter vector: W1[32][33][3][3], b1[32], W2[64][32][3][3], b2[64], W3[32][64][3][3],
// b3[32], w4[32], b4
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + 32 * 33 * 9, OFF_W2 = OFF_B1 + 32, OFF_B2 = OFF_W2 + 64 * 32 * 9,
              OFF_W3 = OFF_B2 + 64, OFF_B3 = OFF_W3 + 32 * 64 * 9, OFF_W4 = OFF_B3 + 32, OFF_B4 = OFF_W4 + 32;
static_assert(OFF_B4 + 1 == NBSI_NET_NPARAM, "parameter count");

// scale slots: the gradient scale that entered layer l's weight gradient is slot l
constexpr int N_SCALE = 4;

__device__ __forceinline__ int acc_row(int r, int lane) { return (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3); }

// 2^e with x * 2^e in [2^11, 2^12) (1 when x is 0 or not finite): the gradient's largest
// magnitude lands just below 2^12, far inside FP16's range, with 2^12 of headroom for the
// sums of the next product
__device__ __forceinline__ float pow2_scale(float x) {
    if (!(x > 0.f) || !isfinite(x)) return 1.f;
    int ex = 0;
    frexpf(x, &ex);  // x = f 2^ex, f in [0.5, 1)
    ex = max(-100, min(100, 12 - ex));
    return ldexpf(1.f, ex);
}

// ---------------- stamps ----------------
__global__ __launch_bounds__(256) void stamps_kernel(const float *__restrict__ cube, int n_chan, int n_pix,
                                                     const nbsi_cand *__restrict__ cands, int n,
                                                     _Float16 *__restrict__ out) {
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long)n * SC * NPOS) return;
    const int k = (int)(e / (SC * NPOS)), rem = (int)(e % (SC * NPOS));
    const int dc = rem / NPOS, p = rem % NPOS;
    const nbsi_cand cd = cands[k];
    const int c = cd.c + dc - HALF_C, y = cd.y + p / SP - HALF_P, x = cd.x + p % SP - HALF_P;
    float v = 0.f;
    if (c >= 0 && c < n_chan && y >= 0 && y < n_pix && x >= 0 && x < n_pix)
        v = cube[((size_t)c * n_pix + y) * n_pix + x];
    out[e] = (_Float16)fminf(fmaxf(v, -65504.f), 65504.f);
}

// ---------------- forward ----------------
// One wave per 32 x 32 tile of (row, output channel); four waves per workgroup stack along rows.
template <int CIN, int CINP, int COUT, bool IN_STAMP, bool OUT_F32>
__global__ __launch_bounds__(256) void conv_fwd_kernel(const _Float16 *__restrict__ in, const int *__restrict__ index,
                                                       int n_stamps, int n, const _Float16 *__restrict__ w16,
                                                       const float *__restrict__ bias, void *__restrict__ out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int M = n * NPOS;
    const int m0 = (blockIdx.x * 4 + wave) * 32;
    if (m0 >= M) return;  // uniform per wave; the kernel has no barriers
    const int co0 = blockIdx.y * 32;
    const int i = lane & 31, kq = (lane >> 5) * 8;
    const int m = m0 + i;
    const bool mv = m < M;
    const int b = mv ? m / NPOS : 0, p = mv ? m % NPOS : 0;
    const int y = p / SP, x = p % SP;
    const _Float16 *src = nullptr;
    bool sv = mv;
    if constexpr (IN_STAMP) {
        const int s = index ? index[b] : b;
        sv = mv && s >= 0 && s < n_stamps;
        src = in + (size_t)(sv ? s : 0) * SC * NPOS;
    } else {
        src = in + (size_t)b * NPOS * CINP;
    }
    const _Float16 *wrow = w16 + (size_t)(co0 + i) * 9 * CINP;
    v16f acc;
#pragma unroll
    for (int r = 0; r < 16; r++) acc[r] = 0.f;
    for (int tap = 0; tap < 9; tap++) {
        const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
        const bool ok = sv && yy >= 0 && yy < SP && xx >= 0 && xx < SP;
        const int pp = ok ? yy * SP + xx : 0;
#pragma unroll
        for (int c0 = 0; c0 < CINP; c0 += 16) {
            const int ci = c0 + kq;
            v8h a = {0, 0, 0, 0, 0, 0, 0, 0};
            if (ok) {
                if constexpr (IN_STAMP) {
#pragma unroll
                    for (int e = 0; e < 8; e++) a[e] = (ci + e < CIN) ? src[(ci + e) * NPOS + pp] : (_Float16)0;
                } else {
                    a = *reinterpret_cast<const v8h *>(src + pp * CINP + ci);
                }
            }
            const v8h w = *reinterpret_cast<const v8h *>(wrow + tap * CINP + ci);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, w, acc, 0, 0, 0);
        }
    }
    const int co = co0 + i;
    const float bc = bias[co];
#pragma unroll
    for (int r = 0; r < 16; r++) {
        const int mm = m0 + acc_row(r, lane);
        if (mm >= M) continue;
        const float z = fmaxf(acc[r] + bc, 0.f);
        if constexpr (OUT_F32) reinterpret_cast<float *>(out)[(size_t)mm * COUT + co] = z;
        else reinterpret_cast<_Float16 *>(out)[(size_t)mm * COUT + co] = (_Float16)z;
    }
}

// Global average pool, linear unit, and (with labels) the loss terms and dL/dz = (sigmoid(z) - y) / n.
// 32 lanes per stamp, one per feature.
__global__ __launch_bounds__(256) void head_kernel(const float *__restrict__ a3, int n, const float *__restrict__ theta,
                                                   const float *__restrict__ labels, const int *__restrict__ index,
                                                   int n_stamps, float *__restrict__ feat, float *__restrict__ logits,
                                                   float *__restrict__ dz, float *__restrict__ lossb) {
    const int t = threadIdx.x, b = blockIdx.x * 8 + (t >> 5), c = t & 31;
    const bool bv = b < n;
    float f = 0.f;
    if (bv) {
        for (int p = 0; p < NPOS; p++) f += a3[((size_t)b * NPOS + p) * 32 + c];
        f = f / (float)NPOS;
    }
    float s = bv ? theta[OFF_W4 + c] * f : 0.f;
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o, 32);
    if (!bv) return;
    if (feat) feat[b * 32 + c] = f;
    if (c != 0) return;
    const float z = s + theta[OFF_B4];
    logits[b] = z;
    if (labels) {
        int si = index ? index[b] : b;
        si = (si >= 0 && si < n_stamps) ? si : 0;
        const float yv = labels[si];
        const float sp = fmaxf(z, 0.f) + log1pf(expf(-fabsf(z)));  // log(1 + e^z)
        const float sg = z >= 0.f ? 1.f / (1.f + expf(-z)) : expf(z) / (1.f + expf(z));
        lossb[b] = sp - yv * z;
        dz[b] = (sg - yv) / (float)n;
    }
}

// One workgroup: dL/dw4, dL/db4, the mean loss, and the first gradient scale.
__global__ __launch_bounds__(256) void head_reduce_kernel(const float *__restrict__ feat, const float *__restrict__ dz,
                                                          const float *__restrict__ lossb, int n,
                                                          const float *__restrict__ theta, float *__restrict__ grad,
                                                          float *__restrict__ loss, float *__restrict__ scale) {
    __shared__ float r_w[8][32], r_d[8], r_l[8], r_m[8];
    const int t = threadIdx.x, c = t & 31, j = t >> 5;
    float sw = 0.f, sd = 0.f, sl = 0.f, mx = 0.f;
    // (unrolled so that the loads are issued ahead of the in-order sums)
#pragma unroll 8
    for (int b = j; b < n; b += 8) {
        const float d = dz[b];
        sw += d * feat[b * 32 + c];
        if (c == 0) {
            sd += d;
            sl += lossb[b];
            mx = fmaxf(mx, fabsf(d));
        }
    }
    r_w[j][c] = sw;
    if (c == 0) {
        r_d[j] = sd;
        r_l[j] = sl;
        r_m[j] = mx;
    }
    __syncthreads();
    if (t < 32) {
        float s = 0.f;
        for (int q = 0; q < 8; q++) s += r_w[q][t];
        grad[OFF_W4 + t] = s;
    }
    if (t == 0) {
        float d = 0.f, l = 0.f, m = 0.f, mw = 0.f;
        for (int q = 0; q < 8; q++) {
            d += r_d[q];
            l += r_l[q];
            m = fmaxf(m, r_m[q]);
        }
        for (int q = 0; q < 32; q++) mw = fmaxf(mw, fabsf(theta[OFF_W4 + q]));
        grad[OFF_B4] = d;
        if (loss) loss[0] = l / (float)n;
        // |dL/dA3| <= max|dz| max|w4| / 81 bounds the third layer's output gradient
        scale[3] = pow2_scale(m * mw / (float)NPOS);
    }
}

// dL/dZ3 = dz_b w4[c] / 81 where the third layer's output is positive, scaled, in FP16.
__global__ __launch_bounds__(256) void dz3_kernel(const float *__restrict__ a3, const float *__restrict__ dz,
                                                  const float *__restrict__ theta, const float *__restrict__ scale,
                                                  int n, _Float16 *__restrict__ dZ) {
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long)n * NPOS * 32) return;
    const int b = (int)(e / (NPOS * 32)), c = (int)(e & 31);
    const float v = dz[b] * theta[OFF_W4 + c] / (float)NPOS;
    dZ[e] = a3[e] > 0.f ? (_Float16)(v * scale[3]) : (_Float16)0;
}

// Weight gradient partials: D[co][k] = sum over this split's rows m of dZ[m][co] X[m (+) tap][ci].
template <int CIN, int CINP, int COUT, bool IN_STAMP>
__global__ __launch_bounds__(256) void wgrad_kernel(const _Float16 *__restrict__ dZ, const _Float16 *__restrict__ in,
                                                    const int *__restrict__ index, int n_stamps, int n, int chunk,
                                                    float *__restrict__ partial) {
    constexpr int K = 9 * CINP;
    constexpr int KT = (K + 31) / 32;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tile = blockIdx.x * 4 + wave;
    if (tile >= (COUT / 32) * KT) return;  // uniform per wave; no barriers
    const int co0 = (tile / KT) * 32, k0 = (tile % KT) * 32;
    const int split = blockIdx.y;
    const int M = n * NPOS;
    const int mb = split * chunk, me = min(M, mb + chunk);
    const int i = lane & 31, kq = (lane >> 5) * 8;
    const int k = k0 + i;
    const bool kv = k < K;
    const int tap = kv ? k / CINP : 0, ci = kv ? k % CINP : 0;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const bool civ = kv && ci < CIN;
    v16f acc;
#pragma unroll
    for (int r = 0; r < 16; r++) acc[r] = 0.f;
    for (int m = mb; m < me; m += 16) {
        v8h a, xb;
        // the lane's 8 rows lie in at most two stamps: their indices are read once
        int s_lo = 0, s_hi = 0;
        const int b_lo = (m + kq) / NPOS;
        if constexpr (IN_STAMP) {
            s_lo = index ? (b_lo < n ? index[b_lo] : -1) : b_lo;
            s_hi = index ? (b_lo + 1 < n ? index[b_lo + 1] : -1) : b_lo + 1;
        }
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int mm = m + kq + e;
            const bool ok = mm < me;
            a[e] = ok ? dZ[(size_t)mm * COUT + co0 + i] : (_Float16)0;
            _Float16 xv = 0;
            if (ok && civ) {
                const int b = mm / NPOS, p = mm % NPOS;
                const int yy = p / SP + dy, xx = p % SP + dx;
                if (yy >= 0 && yy < SP && xx >= 0 && xx < SP) {
                    if constexpr (IN_STAMP) {
                        const int s = b == b_lo ? s_lo : s_hi;
                        if (s >= 0 && s < n_stamps) xv = in[((size_t)s * SC + ci) * NPOS + yy * SP + xx];
                    } else {
                        xv = in[((size_t)b * NPOS + yy * SP + xx) * CINP + ci];
                    }
                }
            }
            xb[e] = xv;
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, xb, acc, 0, 0, 0);
    }
    if (!kv) return;
#pragma unroll
    for (int r = 0; r < 16; r++) partial[((size_t)split * COUT + co0 + acc_row(r, lane)) * K + k] = acc[r];
}

// Sum the partials, undo the gradient scale, write the oracle layout [o][i][dy][dx].  A
// workgroup takes 64 consecutive (co, k) of the partials' own layout (contiguous reads); its
// four waves sum the splits q = w, w + 4, ... and are then added in wave order, so the result
// is deterministic.  Padded input channels (ci >= cin) are skipped.
__global__ __launch_bounds__(256) void wgrad_reduce_kernel(const float *__restrict__ partial, int ksplit, int cout,
                                                           int cin, int cinp, const float *__restrict__ scale, int slot,
                                                           float *__restrict__ grad, int off) {
    __shared__ float red[4][64];
    const int K = 9 * cinp;
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int e = blockIdx.x * 64 + l;
    const bool ev = e < cout * K;
    float s = 0.f;
    if (ev) {
        // (unrolled so that the loads are issued ahead of the in-order additions)
#pragma unroll 8
        for (int q = w; q < ksplit; q += 4) s += partial[(size_t)q * cout * K + e];
    }
    red[w][l] = s;
    __syncthreads();
    if (w != 0 || !ev) return;
    const int co = e / K, k = e % K, tap = k / cinp, ci = k % cinp;
    if (ci >= cin) return;
    const float a = ((red[0][l] + red[1][l]) + red[2][l]) + red[3][l];
    grad[off + (co * cin + ci) * 9 + tap] = a / scale[slot];
}

// Bias gradient, first level: workgroup q sums dZ over its rows [q rows, (q + 1) rows).  A
// thread reads 8 channels of a row with one 16-byte load; the row lanes of each channel are
// summed in a fixed order, so the result is deterministic.
template <int COUT>
__global__ __launch_bounds__(256) void bgrad_partial_kernel(const _Float16 *__restrict__ dZ, int M, int rows,
                                                            float *__restrict__ partial) {
    constexpr int CG = COUT / 8, RL = 256 / CG;  // 8-channel groups per row, row lanes
    static_assert(COUT % 8 == 0 && 256 % CG == 0, "whole 16-byte groups");
    __shared__ float red[RL][COUT + 1];
    const int t = threadIdx.x, g = t % CG, rl = t / CG;
    const int m0 = blockIdx.x * rows, m1 = min(M, m0 + rows);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int m = m0 + rl; m < m1; m += RL) {
        const v8h x = *reinterpret_cast<const v8h *>(dZ + (size_t)m * COUT + 8 * g);
#pragma unroll
        for (int i = 0; i < 8; i++) s[i] += (float)x[i];
    }
#pragma unroll
    for (int i = 0; i < 8; i++) red[rl][8 * g + i] = s[i];
    __syncthreads();
    if (t < COUT) {
        float a = 0.f;
        for (int r = 0; r < RL; r++) a += red[r][t];
        partial[(size_t)blockIdx.x * COUT + t] = a;
    }
}

// Bias gradient, second level: each channel's partials over RL lanes, the lanes in a fixed
// order, the gradient scale undone.
template <int COUT>
__global__ __launch_bounds__(256) void bgrad_final_kernel(const float *__restrict__ partial, int n_part,
                                                          const float *__restrict__ scale, int slot,
                                                          float *__restrict__ grad, int off) {
    constexpr int RL = 256 / COUT;
    __shared__ float red[256];
    const int t = threadIdx.x, co = t % COUT, rl = t / COUT;
    float s = 0.f;
#pragma unroll 8
    for (int q = rl; q < n_part; q += RL) s += partial[(size_t)q * COUT + co];
    red[t] = s;
    __syncthreads();
    if (t < COUT) {
        float a = 0.f;
#pragma unroll
        for (int r = 0; r < RL; r++) a += red[r * COUT + t];
        grad[off + t] = a / scale[slot];
    }
}

// Data gradient of a convolution, masked by the previous ReLU:
// dA[m][ci] = [A_prev[m][ci] > 0] sum_{tap, co} dZ[m (-) tap][co] W[co][ci][tap],
// with W read transposed as WT[ci][tap][co].  Also the largest |dA| (as an ordered integer).
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void dgrad_kernel(const _Float16 *__restrict__ dZ, const _Float16 *__restrict__ wt,
                                                    const _Float16 *__restrict__ a_prev, int n, float *__restrict__ dA,
                                                    unsigned *__restrict__ maxbits) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int M = n * NPOS;
    const int m0 = (blockIdx.x * 4 + wave) * 32;
    if (m0 >= M) return;  // uniform per wave; no barriers
    const int ci0 = blockIdx.y * 32;
    const int i = lane & 31, kq = (lane >> 5) * 8;
    const int m = m0 + i;
    const bool mv = m < M;
    const int b = mv ? m / NPOS : 0, p = mv ? m % NPOS : 0;
    const int y = p / SP, x = p % SP;
    const _Float16 *wrow = wt + (size_t)(ci0 + i) * 9 * COUT;
    v16f acc;
#pragma unroll
    for (int r = 0; r < 16; r++) acc[r] = 0.f;
    for (int tap = 0; tap < 9; tap++) {
        // Z[q] met this position through tap (dy, dx) when q = (y - dy + 1, x - dx + 1)
        const int qy = y - (tap / 3 - 1), qx = x - (tap % 3 - 1);
        const bool ok = mv && qy >= 0 && qy < SP && qx >= 0 && qx < SP;
        const _Float16 *zrow = dZ + ((size_t)b * NPOS + (ok ? qy * SP + qx : 0)) * COUT;
#pragma unroll
        for (int c0 = 0; c0 < COUT; c0 += 16) {
            const int cc = c0 + kq;
            v8h a = {0, 0, 0, 0, 0, 0, 0, 0};
            if (ok) a = *reinterpret_cast<const v8h *>(zrow + cc);
            const v8h w = *reinterpret_cast<const v8h *>(wrow + tap * COUT + cc);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, w, acc, 0, 0, 0);
        }
    }
    const int c = ci0 + i;
    float mx = 0.f;
#pragma unroll
    for (int r = 0; r < 16; r++) {
        const int mm = m0 + acc_row(r, lane);
        if (mm >= M) continue;
        const float v = (float)a_prev[(size_t)mm * CIN + c] > 0.f ? acc[r] : 0.f;
        dA[(size_t)mm * CIN + c] = v;
        mx = fmaxf(mx, fabsf(v));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if (lane == 0) atomicMax(maxbits, __float_as_uint(mx));  // ordered like the values (non-negative)
}

// dZ (FP16) = dA times the power of two that brings max |dA| below 2^12; records the new scale.
__global__ __launch_bounds__(256) void dz_convert_kernel(const float *__restrict__ dA, long n_elem,
                                                         const unsigned *__restrict__ maxbits,
                                                         float *__restrict__ scale, int slot_in, int slot_out,
                                                         _Float16 *__restrict__ dZ) {
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    const float f = pow2_scale(__uint_as_float(*maxbits));
    if (e == 0) scale[slot_out] = scale[slot_in] * f;
    if (e < n_elem) dZ[e] = (_Float16)(dA[e] * f);
}

__global__ void fill_u32_kernel(unsigned *p, int n, unsigned v) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

// FP16 copies of the convolution weights: W16[co][tap][ci (padded)] and WT16[ci][tap][co].
__global__ __launch_bounds__(256) void pack_weights_kernel(const float *__restrict__ w, int cout, int cin, int cinp,
                                                           _Float16 *__restrict__ w16, _Float16 *__restrict__ wt16) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < cout * 9 * cinp) {
        const int co = e / (9 * cinp), rem = e % (9 * cinp), tap = rem / cinp, ci = rem % cinp;
        w16[e] = ci < cin ? (_Float16)w[(co * cin + ci) * 9 + tap] : (_Float16)0;
    }
    if (wt16 && e < cin * 9 * cout) {
        const int ci = e / (9 * cout), rem = e % (9 * cout), tap = rem / cout, co = rem % cout;
        wt16[e] = (_Float16)w[(co * cin + ci) * 9 + tap];
    }
}

__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ theta, float *__restrict__ m,
                                                   float *__restrict__ v, const float *__restrict__ g, int n, float lr,
                                                   float b1, float b2, float eps, float c1, float c2) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.f - b1) * gi;
    const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    theta[e] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

inline unsigned blocks(long n, int per = 256) { return (unsigned)((n + per - 1) / per); }

}  // namespace

struct nbsi_net {
    nbsi_ctx *ctx = nullptr;
    int device = 0, max_batch = 0;
    long step = 0;
    std::vector<void *> owned;
    float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *scale = nullptr;
    float *feat = nullptr, *logits = nullptr, *dz = nullptr, *lossb = nullptr, *a3 = nullptr, *dA = nullptr,
          *partial = nullptr;
    unsigned *maxbits = nullptr;
    _Float16 *w16[3] = {}, *wt16[3] = {}, *a1 = nullptr, *a2 = nullptr, *dZ = nullptr;
    bool packed = false;
};

namespace {

constexpr int MAX_KSPLIT = 256;
constexpr int BIAS_PARTS = 256;  // workgroups of the bias gradient's first level
constexpr size_t PARTIAL_FLOATS = (size_t)MAX_KSPLIT * 64 * 9 * 64;

template <typename T>
int net_alloc(nbsi_net *net, size_t count, T **out) {
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(256, count * sizeof(T))) != hipSuccess) return NBSI_ENOMEM;
    net->owned.push_back(p);
    *out = (T *)p;
    return NBSI_OK;
}

void net_free(nbsi_net *net) {
    if (net->ctx) (void)hipStreamSynchronize(net->ctx->stream);
    for (void *p : net->owned) (void)hipFree(p);
    delete net;
}

struct NetDevice {  // current-device guard
    int prev = -1, dev;
    explicit NetDevice(int d) : dev(d) {
        (void)hipGetDevice(&prev);
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~NetDevice() {
        if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
    }
};

hipError_t pack_weights(nbsi_net *net, hipStream_t st) {
    const int dims[3][3] = {{33, 48, 32}, {32, 32, 64}, {64, 64, 32}};
    const int offs[3] = {OFF_W1, OFF_W2, OFF_W3};
    for (int l = 0; l < 3; l++) {
        const int cin = dims[l][0], cinp = dims[l][1], cout = dims[l][2];
        const long n = std::max((long)cout * 9 * cinp, (long)cin * 9 * cout);
        hipLaunchKernelGGL(pack_weights_kernel, dim3(blocks(n)), dim3(256), 0, st, net->theta + offs[l], cout, cin,
                           cinp, net->w16[l], net->wt16[l]);
    }
    net->packed = true;
    return hipGetLastError();
}

// Splits of the weight gradient over the batch: about 160 rows each (ten MFMA steps per wave),
// at most MAX_KSPLIT.  Each wave's loop is bound by the latency of its operand loads, so many
// short splits run faster than few long ones (at batch 512: 256 splits 1.56M stamps/s of
// training, 64 splits 1.25M; 384 and 512 splits were slower again, their partial sums costing
// more than they save).
int ksplit_for(int M) { return std::max(1, std::min(MAX_KSPLIT, M / 160)); }

// Forward pass; with labels also the head's loss terms and dL/dz.
hipError_t forward(nbsi_net *net, const uint16_t *stamps, int n_stamps, const int32_t *index, const float *labels,
                   int n, float *logits, hipStream_t st) {
    hipError_t e = hipSuccess;
    if (!net->packed && (e = pack_weights(net, st)) != hipSuccess) return e;
    const _Float16 *x = reinterpret_cast<const _Float16 *>(stamps);
    const int M = n * NPOS;
    const dim3 blk(256);
    hipLaunchKernelGGL((conv_fwd_kernel<33, 48, 32, true, false>), dim3(blocks(M, 128), 1), blk, 0, st, x, index,
                       n_stamps, n, net->w16[0], net->theta + OFF_B1, (void *)net->a1);
    hipLaunchKernelGGL((conv_fwd_kernel<32, 32, 64, false, false>), dim3(blocks(M, 128), 2), blk, 0, st,
                       (const _Float16 *)net->a1, nullptr, 0, n, net->w16[1], net->theta + OFF_B2, (void *)net->a2);
    hipLaunchKernelGGL((conv_fwd_kernel<64, 64, 32, false, true>), dim3(blocks(M, 128), 1), blk, 0, st,
                       (const _Float16 *)net->a2, nullptr, 0, n, net->w16[2], net->theta + OFF_B3, (void *)net->a3);
    hipLaunchKernelGGL(head_kernel, dim3(blocks(n, 8)), blk, 0, st, net->a3, n, net->theta, labels, index, n_stamps,
                       net->feat, logits, net->dz, net->lossb);
    return hipGetLastError();
}

template <int CIN, int CINP, int COUT, bool IN_STAMP>
void weight_grads(nbsi_net *net, const _Float16 *x, const int32_t *index, int n_stamps, int n, int slot, int off_w,
                  int off_b, float *grad, hipStream_t st) {
    const int M = n * NPOS;
    const int ks = ksplit_for(M);
    const int chunk = (M + ks - 1) / ks;
    constexpr int KT = (9 * CINP + 31) / 32;
    hipLaunchKernelGGL((wgrad_kernel<CIN, CINP, COUT, IN_STAMP>), dim3(blocks((COUT / 32) * KT, 4), ks), dim3(256), 0,
                       st, (const _Float16 *)net->dZ, x, index, n_stamps, n, chunk, net->partial);
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(blocks(COUT * 9 * CINP, 64)), dim3(256), 0, st, net->partial, ks, COUT,
                       CIN, CINP, net->scale, slot, grad, off_w);
    // the bias partials (up to BIAS_PARTS per channel) reuse the weight partials' buffer, which
    // the reduction above has read
    static_assert(256 % COUT == 0 && (size_t)BIAS_PARTS * COUT <= PARTIAL_FLOATS, "bias partials");
    const int n_part = std::max(1, std::min(BIAS_PARTS, M / 64));
    const int rows = (M + n_part - 1) / n_part;
    hipLaunchKernelGGL(bgrad_partial_kernel<COUT>, dim3(n_part), dim3(256), 0, st, (const _Float16 *)net->dZ, M, rows,
                       net->partial);
    hipLaunchKernelGGL(bgrad_final_kernel<COUT>, dim3(1), dim3(256), 0, st, net->partial, n_part, net->scale, slot,
                       grad, off_b);
}

// Backward pass after forward(..., labels): every parameter's gradient into grad.
hipError_t backward(nbsi_net *net, const uint16_t *stamps, int n_stamps, const int32_t *index, int n, float *loss,
                    float *grad, hipStream_t st) {
    const int M = n * NPOS;
    const dim3 blk(256);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, net->maxbits, 2, 0u);
    hipLaunchKernelGGL(head_reduce_kernel, dim3(1), blk, 0, st, net->feat, net->dz, net->lossb, n, net->theta, grad,
                       loss, net->scale);
    hipLaunchKernelGGL(dz3_kernel, dim3(blocks((long)M * 32)), blk, 0, st, net->a3, net->dz, net->theta, net->scale, n,
                       net->dZ);
    // layer 3 (input a2, 64 -> 32)
    weight_grads<64, 64, 32, false>(net, net->a2, nullptr, 0, n, 3, OFF_W3, OFF_B3, grad, st);
    hipLaunchKernelGGL((dgrad_kernel<64, 32>), dim3(blocks(M, 128), 2), blk, 0, st, (const _Float16 *)net->dZ,
                       (const _Float16 *)net->wt16[2], (const _Float16 *)net->a2, n, net->dA, net->maxbits);
    hipLaunchKernelGGL(dz_convert_kernel, dim3(blocks((long)M * 64)), blk, 0, st, net->dA, (long)M * 64, net->maxbits,
                       net->scale, 3, 2, net->dZ);
    // layer 2 (input a1, 32 -> 64)
    weight_grads<32, 32, 64, false>(net, net->a1, nullptr, 0, n, 2, OFF_W2, OFF_B2, grad, st);
    hipLaunchKernelGGL((dgrad_kernel<32, 64>), dim3(blocks(M, 128), 1), blk, 0, st, (const _Float16 *)net->dZ,
                       (const _Float16 *)net->wt16[1], (const _Float16 *)net->a1, n, net->dA, net->maxbits + 1);
    hipLaunchKernelGGL(dz_convert_kernel, dim3(blocks((long)M * 32)), blk, 0, st, net->dA, (long)M * 32,
                       net->maxbits + 1, net->scale, 2, 1, net->dZ);
    // layer 1 (input: the stamps, 33 -> 32)
    weight_grads<33, 48, 32, true>(net, reinterpret_cast<const _Float16 *>(stamps), index, n_stamps, n, 1, OFF_W1,
                                   OFF_B1, grad, st);
    return hipGetLastError();
}

int check_batch(nbsi_net *net, const uint16_t *stamps, int n_stamps, int n) {
    if (!stamps || n < 1 || n > net->max_batch || n_stamps < 1) return NBSI_EINVAL;
    if ((uintptr_t)stamps & 7u) return NBSI_EINVAL;
    return NBSI_OK;
}

int check_index(const int32_t *index, int n_stamps, int n) { return (!index && n > n_stamps) ? NBSI_EINVAL : NBSI_OK;
}

}  // namespace

extern "C" {

int nbsi_stamps(nbsi_ctx *ctx, const float *cube, int n_chan, int n_pix, const nbsi_cand *cands, int n,
                uint16_t *stamps) {
    if (!ctx) return NBSI_EINVAL;
    if (n == 0) return NBSI_OK;
    if (!cube || !cands || !stamps || n < 0 || n_chan < 1 || n_pix < 1 || (long)n * SC * NPOS > (1L << 31))
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_stamps: bad arguments");
    NetDevice g(ctx->device);
    hipLaunchKernelGGL(stamps_kernel, dim3(blocks((long)n * SC * NPOS)), dim3(256), 0, ctx->stream, cube, n_chan,
                       n_pix, cands, n, reinterpret_cast<_Float16 *>(stamps));
    if (hipGetLastError() != hipSuccess) return nbsi_fail(ctx, NBSI_EHIP, "nbsi_stamps: launch failed");
    return NBSI_OK;
}

int nbsi_net_create(nbsi_ctx *ctx, const float *params_host, int max_batch, nbsi_net **out) {
    if (!ctx || !out) return NBSI_EINVAL;
    *out = nullptr;
    if (!params_host || max_batch < 1 || max_batch > NBSI_NET_MAX_BATCH)
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_net_create: bad arguments");
    NetDevice g(ctx->device);
    nbsi_net *net = new (std::nothrow) nbsi_net();
    if (!net) return NBSI_ENOMEM;
    net->ctx = ctx;
    net->device = ctx->device;
    net->max_batch = max_batch;
    const size_t B = max_batch, P = NBSI_NET_NPARAM;
    int rc = NBSI_OK;
    rc = rc ? rc : net_alloc(net, P, &net->theta);
    rc = rc ? rc : net_alloc(net, P, &net->m);
    rc = rc ? rc : net_alloc(net, P, &net->v);
    rc = rc ? rc : net_alloc(net, P, &net->grad);
    rc = rc ? rc : net_alloc(net, (size_t)N_SCALE, &net->scale);
    rc = rc ? rc : net_alloc(net, B * 32, &net->feat);
    rc = rc ? rc : net_alloc(net, B, &net->logits);
    rc = rc ? rc : net_alloc(net, B, &net->dz);
    rc = rc ? rc : net_alloc(net, B, &net->lossb);
    rc = rc ? rc : net_alloc(net, B * NPOS * 32, &net->a3);
    rc = rc ? rc : net_alloc(net, B * NPOS * 64, &net->dA);
    rc = rc ? rc : net_alloc(net, PARTIAL_FLOATS, &net->partial);
    rc = rc ? rc : net_alloc(net, (size_t)2, &net->maxbits);
    rc = rc ? rc : net_alloc(net, B * NPOS * 32, &net->a1);
    rc = rc ? rc : net_alloc(net, B * NPOS * 64, &net->a2);
    rc = rc ? rc : net_alloc(net, B * NPOS * 64, &net->dZ);
    rc = rc ? rc : net_alloc(net, (size_t)32 * 9 * 48, &net->w16[0]);
    rc = rc ? rc : net_alloc(net, (size_t)64 * 9 * 32, &net->w16[1]);
    rc = rc ? rc : net_alloc(net, (size_t)32 * 9 * 64, &net->w16[2]);
    rc = rc ? rc : net_alloc(net, (size_t)33 * 9 * 32, &net->wt16[0]);
    rc = rc ? rc : net_alloc(net, (size_t)32 * 9 * 64, &net->wt16[1]);
    rc = rc ? rc : net_alloc(net, (size_t)64 * 9 * 32, &net->wt16[2]);
    if (rc) {
        net_free(net);
        return nbsi_fail(ctx, rc, "nbsi_net_create: out of device memory");
    }
    *out = net;
    rc = nbsi_net_set_params(net, params_host);
    if (rc) {
        net_free(net);
        *out = nullptr;
        return rc;
    }
    return NBSI_OK;
}

int nbsi_net_destroy(nbsi_net *net) {
    if (!net) return NBSI_EINVAL;
    NetDevice g(net->device);
    net_free(net);
    return NBSI_OK;
}

int nbsi_net_set_params(nbsi_net *net, const float *params_host) {
    if (!net || !params_host) return NBSI_EINVAL;
    NetDevice g(net->device);
    hipStream_t st = net->ctx->stream;
    const size_t bytes = sizeof(float) * NBSI_NET_NPARAM;
    if (hipMemcpyAsync(net->theta, params_host, bytes, hipMemcpyHostToDevice, st) != hipSuccess)
        return nbsi_fail(net->ctx, NBSI_EHIP, "nbsi_net_set_params: copy failed");
    hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks(NBSI_NET_NPARAM)), dim3(256), 0, st, (unsigned *)net->m,
                       NBSI_NET_NPARAM, 0u);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks(NBSI_NET_NPARAM)), dim3(256), 0, st, (unsigned *)net->v,
                       NBSI_NET_NPARAM, 0u);
    net->step = 0;
    if (pack_weights(net, st) != hipSuccess) return nbsi_fail(net->ctx, NBSI_EHIP, "nbsi_net_set_params: launch failed");
    // the host buffer may be reused by the caller as soon as this returns
    if (hipStreamSynchronize(st) != hipSuccess) return nbsi_fail(net->ctx, NBSI_EHIP, "nbsi_net_set_params: sync failed");
    return NBSI_OK;
}

int nbsi_net_get_params(nbsi_net *net, float *params_host) {
    if (!net || !params_host) return NBSI_EINVAL;
    NetDevice g(net->device);
    hipStream_t st = net->ctx->stream;
    if (hipMemcpyAsync(params_host, net->theta, sizeof(float) * NBSI_NET_NPARAM, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return nbsi_fail(net->ctx, NBSI_EHIP, "nbsi_net_get_params: copy failed");
    return NBSI_OK;
}

int nbsi_net_forward(nbsi_net *net, const uint16_t *stamps, int n_stamps, const int32_t *index, int n, float *logits) {
    if (!net) return NBSI_EINVAL;
    if (check_batch(net, stamps, n_stamps, n) || check_index(index, n_stamps, n) || !logits)
        return nbsi_fail(net->ctx, NBSI_EINVAL, "nbsi_net_forward: bad arguments");
    NetDevice g(net->device);
    if (forward(net, stamps, n_stamps, index, nullptr, n, logits, net->ctx->stream) != hipSuccess)
        return nbsi_fail(net->ctx, NBSI_EHIP, "nbsi_net_forward: launch failed");
    return NBSI_OK;
}

int nbsi_net_grad(nbsi_net *net, const uint16_t *stamps, int n_stamps, const int32_t *index, const float *labels, int n,
                  float *loss, float *grad) {
    if (!net) return NBSI_EINVAL;
    if (check_batch(net, stamps, n_stamps, n) || check_index(index, n_stamps, n) || !labels)
        return nbsi_fail(net->ctx, NBSI_EINVAL, "nbsi_net_grad: bad arguments");
    NetDevice g(net->device);
    hipStream_t st = net->ctx->stream;
    float *gout = grad ? grad : net->grad;
    if (forward(net, stamps, n_stamps, index, labels, n, net->logits, st) != hipSuccess ||
        backward(net, stamps, n_stamps, index, n, loss, gout, st) != hipSuccess)
        return nbsi_fail(net->ctx, NBSI_EHIP, "nbsi_net_grad: launch failed");
    return NBSI_OK;
}

int nbsi_net_adam(nbsi_net *net, const float *grad, float lr, float beta1, float beta2, float eps) {
    if (!net) return NBSI_EINVAL;
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f))
        return nbsi_fail(net->ctx, NBSI_EINVAL, "nbsi_net_adam: bad hyper-parameters");
    NetDevice g(net->device);
    hipStream_t st = net->ctx->stream;
    net->step++;
    const double c1 = 1.0 / (1.0 - pow((double)beta1, (double)net->step));
    const double c2 = 1.0 / (1.0 - pow((double)beta2, (double)net->step));
    hipLaunchKernelGGL(adam_kernel, dim3(blocks(NBSI_NET_NPARAM)), dim3(256), 0, st, net->theta, net->m, net->v,
                       grad ? grad : net->grad, NBSI_NET_NPARAM, lr, beta1, beta2, eps, (float)c1, (float)c2);
    if (pack_weights(net, st) != hipSuccess) return nbsi_fail(net->ctx, NBSI_EHIP, "nbsi_net_adam: launch failed");
    return NBSI_OK;
}

int nbsi_net_train_step(nbsi_net *net, const uint16_t *stamps, int n_stamps, const int32_t *index, const float *labels,
                        int n, float lr, float *loss) {
    int rc = nbsi_net_grad(net, stamps, n_stamps, index, labels, n, loss, nullptr);
    if (rc) return rc;
    return nbsi_net_adam(net, nullptr, lr, 0.9f, 0.999f, 1e-8f);
}

}  // extern "C"
