// Device-side complex arithmetic and small-radix DFT butterflies (forward, exp(-2 pi i kn/R)).
#pragma once

#include <hip/hip_runtime.h>

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * (-i)
__device__ __forceinline__ float2 cmul_negi(float2 a) { return make_float2(a.y, -a.x); }
// a * (+i)
__device__ __forceinline__ float2 cmul_posi(float2 a) { return make_float2(-a.y, a.x); }

// Two-level table of exp(-2 pi i j / 2^log_n): W(j) = lo[j & mask] * hi[j >> lo_bits].
// The entries are float32 roundings of float64 values, so every twiddle is within ~1.5 ulp.
struct TwiddleTable {
    const float2 *lo;
    const float2 *hi;
    int lo_bits;
    int mask;
    __device__ __forceinline__ float2 operator()(int j) const {
        return cmul(lo[j & mask], hi[j >> lo_bits]);
    }
};

// Fill a two-level table for n = 2^log_n in LDS (lo_bits = ceil(log_n / 2)).
__device__ __forceinline__ TwiddleTable build_twiddles(float2 *lo, float2 *hi, int log_n, int tid,
                                                       int nthreads) {
    const int lo_bits = (log_n + 1) >> 1;
    const int n_lo = 1 << lo_bits, n_hi = 1 << (log_n - lo_bits);
    const double inv = -2.0 / (double)(1 << log_n);
    for (int j = tid; j < n_lo + n_hi; j += nthreads) {
        double s, c;
        if (j < n_lo) {
            sincospi(inv * (double)j, &s, &c);
            lo[j] = make_float2((float)c, (float)s);
        } else {
            int jj = j - n_lo;
            sincospi(inv * (double)(jj << lo_bits), &s, &c);
            hi[jj] = make_float2((float)c, (float)s);
        }
    }
    TwiddleTable t{lo, hi, lo_bits, n_lo - 1};
    return t;
}

__device__ __forceinline__ void dft2(float2 &a, float2 &b) {
    float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

// natural-order radix-4: (x0, x1, x2, x3) -> (X0, X1, X2, X3)
__device__ __forceinline__ void dft4(float2 &x0, float2 &x1, float2 &x2, float2 &x3) {
    float2 t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3), t3 = csub(x1, x3);
    x0 = cadd(t0, t2);
    x2 = csub(t0, t2);
    x1 = cadd(t1, cmul_negi(t3));
    x3 = csub(t1, cmul_negi(t3));
}

// radix-8 = 4 x 2: n = 2 n1 + n2, k = k1 + 4 k2.  The twiddles W8^k1 of the odd half enter
// the combining sums as fused multiply-adds: (x + i y) W8 = r (x + y) + i r (y - x), so
// a +- that costs one add per component for x + y (or y - x) and one FMA per output.
__device__ __forceinline__ void dft8(float2 *v) {
    const float r = 0.70710678118654752440f;
    dft4(v[0], v[2], v[4], v[6]);  // n2 = 0 -> y0[k1] at v[2 k1]
    dft4(v[1], v[3], v[5], v[7]);  // n2 = 1 -> y1[k1] at v[2 k1 + 1]
    float2 o[8];
    o[0] = cadd(v[0], v[1]);
    o[4] = csub(v[0], v[1]);
    {  // k1 = 1: y1 W8 = r (s, d)
        const float s = v[3].x + v[3].y, d = v[3].y - v[3].x;
        o[1] = make_float2(fmaf(r, s, v[2].x), fmaf(r, d, v[2].y));
        o[5] = make_float2(fmaf(-r, s, v[2].x), fmaf(-r, d, v[2].y));
    }
    o[2] = cadd(v[4], cmul_negi(v[5]));  // k1 = 2: y1 W8^2 = -i y1
    o[6] = csub(v[4], cmul_negi(v[5]));
    {  // k1 = 3: y1 W8^3 = r (d, -s)
        const float s = v[7].x + v[7].y, d = v[7].y - v[7].x;
        o[3] = make_float2(fmaf(r, d, v[6].x), fmaf(-r, s, v[6].y));
        o[7] = make_float2(fmaf(-r, d, v[6].x), fmaf(r, s, v[6].y));
    }
#pragma unroll
    for (int k = 0; k < 8; k++) v[k] = o[k];
}

// radix-16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2.  The inner twiddles W16^(n2 k1) are folded
// into the second stage's sums as fused multiply-adds: W^2 and W^6 terms are r (x +- y); the
// W^1/W^3 and W^3/W^9 pairs combine into sums c (A + tau B) with c = cos(pi/8) and
// tau = tan(pi/8), so every scaled term costs one FMA to form and one per output.
__device__ __forceinline__ void dft16(float2 *v) {
#pragma unroll
    for (int n2 = 0; n2 < 4; n2++) dft4(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    // element (n2, k1) now sits at v[4 k1 + n2]; output k1 + 4 k2 goes to o[k1 + 4 k2]
    const float c = 0.92387953251128675613f;    // cos(pi/8)
    const float tau = 0.41421356237309504880f;  // tan(pi/8)
    const float r = 0.70710678118654752440f;
    float2 o[16];
    {  // k1 = 0: no twiddles
        float2 a = v[0], b = v[1], cc = v[2], d = v[3];
        dft4(a, b, cc, d);
        o[0] = a;
        o[4] = b;
        o[8] = cc;
        o[12] = d;
    }
    {  // k1 = 1: a = v4, x1 = v5 W^1, x2 = v6 W^2, x3 = v7 W^3
        const float2 a = v[4], p = v[5], q = v[7];
        const float s6 = v[6].x + v[6].y, d6 = v[6].y - v[6].x;
        const float2 t0 = make_float2(fmaf(r, s6, a.x), fmaf(r, d6, a.y));
        const float2 t1 = make_float2(fmaf(-r, s6, a.x), fmaf(-r, d6, a.y));
        const float A = p.x + q.y, B = p.y + q.x, C = p.y - q.x, D = p.x - q.y;
        // x1 + x3 = c (A + tau B, C - tau D), x1 - x3 = c (D + tau C, B - tau A)
        const float2 u2 = make_float2(fmaf(tau, B, A), fmaf(-tau, D, C));
        const float2 u3 = make_float2(fmaf(tau, C, D), fmaf(-tau, A, B));
        o[1] = make_float2(fmaf(c, u2.x, t0.x), fmaf(c, u2.y, t0.y));
        o[9] = make_float2(fmaf(-c, u2.x, t0.x), fmaf(-c, u2.y, t0.y));
        o[5] = make_float2(fmaf(c, u3.y, t1.x), fmaf(-c, u3.x, t1.y));
        o[13] = make_float2(fmaf(-c, u3.y, t1.x), fmaf(c, u3.x, t1.y));
    }
    {  // k1 = 2: a = v8, x1 = v9 W^2, x2 = v10 W^4 = -i v10, x3 = v11 W^6
        const float2 a = v[8], x2 = cmul_negi(v[10]);
        const float2 t0 = cadd(a, x2), t1 = csub(a, x2);
        const float s9 = v[9].x + v[9].y, d9 = v[9].y - v[9].x;
        const float s11 = v[11].x + v[11].y, d11 = v[11].y - v[11].x;
        // x1 = r (s9, d9), x3 = r (d11, -s11)
        const float2 P = make_float2(s9 + d11, d9 - s11), Q = make_float2(s9 - d11, d9 + s11);
        o[2] = make_float2(fmaf(r, P.x, t0.x), fmaf(r, P.y, t0.y));
        o[10] = make_float2(fmaf(-r, P.x, t0.x), fmaf(-r, P.y, t0.y));
        o[6] = make_float2(fmaf(r, Q.y, t1.x), fmaf(-r, Q.x, t1.y));
        o[14] = make_float2(fmaf(-r, Q.y, t1.x), fmaf(r, Q.x, t1.y));
    }
    {  // k1 = 3: a = v12, x1 = v13 W^3, x2 = v14 W^6, x3 = v15 W^9
        const float2 a = v[12], p = v[13], q = v[15];
        const float s14 = v[14].x + v[14].y, d14 = v[14].y - v[14].x;  // x2 = r (d14, -s14)
        const float2 t0 = make_float2(fmaf(r, d14, a.x), fmaf(-r, s14, a.y));
        const float2 t1 = make_float2(fmaf(-r, d14, a.x), fmaf(r, s14, a.y));
        const float A = p.x - q.y, B = p.y - q.x, C = p.y + q.x, D = p.x + q.y;
        // x1 + x3 = (c (B + tau A), -c (D - tau C)), x1 - x3 = (c (C + tau D), -c (A - tau B))
        const float2 u2 = make_float2(fmaf(tau, A, B), fmaf(-tau, C, D));
        const float2 u3 = make_float2(fmaf(tau, D, C), fmaf(-tau, B, A));
        o[3] = make_float2(fmaf(c, u2.x, t0.x), fmaf(-c, u2.y, t0.y));
        o[11] = make_float2(fmaf(-c, u2.x, t0.x), fmaf(c, u2.y, t0.y));
        o[7] = make_float2(fmaf(-c, u3.y, t1.x), fmaf(-c, u3.x, t1.y));
        o[15] = make_float2(fmaf(c, u3.y, t1.x), fmaf(c, u3.x, t1.y));
    }
#pragma unroll
    for (int k = 0; k < 16; k++) v[k] = o[k];
}

template <int R>
__device__ __forceinline__ void dft_r(float2 *v) {
    if constexpr (R == 2) dft2(v[0], v[1]);
    else if constexpr (R == 4) dft4(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8(v);
    else dft16(v);
}

// One Stockham pass on E register elements per thread (E / R butterflies per thread) of an
// L-point transform spread over `nt` threads.  Register v[b*R + r] holds input element
// j + r*L/R with j = t + nt*b; after the pass it holds output element
// (j / ns) * ns * R + (j % ns) + r * ns.  Twiddles W_{ns R}^{(j % ns) r} come from `tw`, a
// table of the 2^log_tab-th roots (log_tab >= log2 L).
template <int R, int E>
__device__ __forceinline__ void stockham_regs(float2 *v, int t, int nt, int log_l, int ns,
                                              const TwiddleTable &tw, int log_tab) {
#pragma unroll
    for (int b = 0; b < E / R; b++) {
        const int j = t + nt * b;
        const int k = j & (ns - 1);
        if (ns > 1) {
            // W_{ns R}^{k r} = W_tab^{k r 2^log_tab / (ns R)}
            const int sh = log_tab - (31 - __clz(ns * R));
#pragma unroll
            for (int r = 1; r < R; r++) v[b * R + r] = cmul(v[b * R + r], tw((k * r) << sh));
        }
        dft_r<R>(v + b * R);
    }
    (void)log_l;
}

// LDS layout of transform buffers: one pad element after every 32, so the strided Stockham
// writes (stride = ns * R elements) spread over the 64 LDS banks instead of piling onto a few.
__device__ __forceinline__ int pidx(int i) { return i + (i >> 5); }
__host__ __device__ constexpr int padded_size(int n) { return n + n / 32; }

// Write the pass outputs of stockham_regs to LDS (row of length L starting at buf).
template <int R, int E>
__device__ __forceinline__ void stockham_store(float2 *buf, const float2 *v, int t, int nt, int ns) {
#pragma unroll
    for (int b = 0; b < E / R; b++) {
        const int j = t + nt * b;
        const int base = (j / ns) * ns * R + (j & (ns - 1));
#pragma unroll
        for (int r = 0; r < R; r++) buf[pidx(base + r * ns)] = v[b * R + r];
    }
}

// Load the inputs of the next pass (radix R) from LDS.
template <int R, int E>
__device__ __forceinline__ void stockham_load(const float2 *buf, float2 *v, int t, int nt, int log_l) {
    const int stride = (1 << log_l) / R;
    // for strides that are multiples of 32 the pad of j + r*stride is pad(j) + r*stride/32, so
    // one base address serves all R loads
    const int pstride = (stride & 31) ? 0 : stride + (stride >> 5);
#pragma unroll
    for (int b = 0; b < E / R; b++) {
        const int j = t + nt * b;
        const int pj = pidx(j);
#pragma unroll
        for (int r = 0; r < R; r++) v[b * R + r] = pstride ? buf[pj + r * pstride] : buf[pidx(j + r * stride)];
    }
}
