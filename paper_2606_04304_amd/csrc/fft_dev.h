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

// radix-8 = 4 x 2: n = 2 n1 + n2, k = k1 + 4 k2
__device__ __forceinline__ void dft8(float2 *v) {
    const float r = 0.70710678118654752440f;
    dft4(v[0], v[2], v[4], v[6]);  // n2 = 0 -> y0[k1]
    dft4(v[1], v[3], v[5], v[7]);  // n2 = 1 -> y1[k1]
    // twiddle y1[k1] *= W8^k1
    v[3] = cmul(v[3], make_float2(r, -r));
    v[5] = cmul_negi(v[5]);
    v[7] = cmul(v[7], make_float2(-r, -r));
    float2 o[8];
#pragma unroll
    for (int k1 = 0; k1 < 4; k1++) {
        float2 a = v[2 * k1], b = v[2 * k1 + 1];
        o[k1] = cadd(a, b);
        o[k1 + 4] = csub(a, b);
    }
#pragma unroll
    for (int k = 0; k < 8; k++) v[k] = o[k];
}

// radix-16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
__device__ __forceinline__ void dft16(float2 *v) {
#pragma unroll
    for (int n2 = 0; n2 < 4; n2++) dft4(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    // element (n2, k1) now sits at v[4 k1 + n2]; twiddle by W16^(n2 k1)
    const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;
    const float r = 0.70710678118654752440f;
    v[4 + 1] = cmul(v[4 + 1], make_float2(c1, -s1));   // k1=1,n2=1: W^1
    v[4 + 2] = cmul(v[4 + 2], make_float2(r, -r));     // W^2
    v[4 + 3] = cmul(v[4 + 3], make_float2(s1, -c1));   // W^3
    v[8 + 1] = cmul(v[8 + 1], make_float2(r, -r));     // k1=2: W^2
    v[8 + 2] = cmul_negi(v[8 + 2]);                    // W^4
    v[8 + 3] = cmul(v[8 + 3], make_float2(-r, -r));    // W^6
    v[12 + 1] = cmul(v[12 + 1], make_float2(s1, -c1)); // k1=3: W^3
    v[12 + 2] = cmul(v[12 + 2], make_float2(-r, -r));  // W^6
    v[12 + 3] = cmul(v[12 + 3], make_float2(-c1, s1)); // W^9
    float2 o[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; k1++) {
        float2 a = v[4 * k1], b = v[4 * k1 + 1], c = v[4 * k1 + 2], d = v[4 * k1 + 3];
        dft4(a, b, c, d);
        o[k1] = a;
        o[k1 + 4] = b;
        o[k1 + 8] = c;
        o[k1 + 12] = d;
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
