// Stage II automated cuts (Sec. 2.4): Gaussian centroid fits of candidate cutouts with
// covariance errors scaled by the reduced chi-square, the synthesized beam from a fit to the
// point-spread function, and flags for extended morphology and deviant image noise.
//
// One wavefront fits one cutout in FP64: each lane holds up to two pixels of the (2h+1)^2 cutout
// (h <= 5), the normal equations (28 + 7 sums) are reduced across the wave with butterflies so
// every lane holds the same totals, and every lane then runs the same 7 x 7 Cholesky solve of the
// Levenberg-Marquardt step.  The work per candidate is tiny next to the imaging that produced the
// cube; the kernel is latency-bound and exists so that the cuts run where the images live.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace {

constexpr int NP = 7;          // amp, x0, y0, a, b, c, bkg
constexpr int S2_WAVES = 1;    // candidates per workgroup (a slow fit holds back no other)
constexpr int LM_MAX_IT = 300;
constexpr double FWHM_PER_SIGMA = 2.3548200450309493;  // 2 sqrt(2 ln 2)

// A lane's double moved across lanes by a DPP pattern (both halves).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Wave sum that leaves the same (bitwise) total in every lane: within rows of 16 lanes by DPP
// (pair swap, quad half swap, half-row mirror, row mirror: each partner holds the other half's
// partial sum), then across rows by lane shuffles.
__device__ __forceinline__ double wsum(double v) {
    v += dpp_move<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x141>(v);  // row_half_mirror
    v += dpp_move<0x140>(v);  // row_mirror
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

// Orders LDS accesses of one wavefront: writes before the call are visible to every lane of the
// wave after it (wavefront-scope fences keep the compiler from moving accesses across).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct Normal {
    double h[28];  // upper triangle of J^T J, row-major
    double g[NP];  // J^T r
    double rss;
};

__device__ __forceinline__ int tri(int i, int j) { return i * NP - i * (i - 1) / 2 + (j - i); }  // i <= j

// Model f = bkg + amp exp(-Q/2), Q = a dx^2 + 2 b dx dy + c dy^2 at the lane's pixels; residual
// r = f - d.  Accumulates the lane's share of J^T J, J^T r and RSS and reduces them over the wave.
__device__ void normal_eq(const double p[NP], const double px[2], const double py[2], const double d[2],
                          const bool on[2], Normal &ne) {
#pragma unroll
    for (int k = 0; k < 28; k++) ne.h[k] = 0.0;
#pragma unroll
    for (int k = 0; k < NP; k++) ne.g[k] = 0.0;
    double rss = 0.0;
#pragma unroll
    for (int s = 0; s < 2; s++) {
        if (!on[s]) continue;
        const double dx = px[s] - p[1], dy = py[s] - p[2];
        const double E = exp(-0.5 * (p[3] * dx * dx + 2.0 * p[4] * dx * dy + p[5] * dy * dy));
        const double AE = p[0] * E;
        const double r = p[6] + AE - d[s];
        double J[NP];
        J[0] = E;
        J[1] = AE * (p[3] * dx + p[4] * dy);
        J[2] = AE * (p[4] * dx + p[5] * dy);
        J[3] = -0.5 * AE * dx * dx;
        J[4] = -AE * dx * dy;
        J[5] = -0.5 * AE * dy * dy;
        J[6] = 1.0;
#pragma unroll
        for (int i = 0; i < NP; i++) {
            ne.g[i] += J[i] * r;
#pragma unroll
            for (int j = i; j < NP; j++) ne.h[tri(i, j)] += J[i] * J[j];
        }
        rss += r * r;
    }
#pragma unroll
    for (int k = 0; k < 28; k++) ne.h[k] = wsum(ne.h[k]);
#pragma unroll
    for (int k = 0; k < NP; k++) ne.g[k] = wsum(ne.g[k]);
    ne.rss = wsum(rss);
}

// In-place Cholesky M = L L^T of a packed symmetric matrix (L stored in the same upper-triangle
// slots, transposed).  False when M is not numerically positive definite.
__device__ bool cholesky(double m[28]) {
#pragma unroll
    for (int j = 0; j < NP; j++) {
        double s = m[tri(j, j)];
#pragma unroll
        for (int k = 0; k < j; k++) s -= m[tri(k, j)] * m[tri(k, j)];
        if (!(s > 0.0)) return false;
        const double l = sqrt(s);
        m[tri(j, j)] = l;
#pragma unroll
        for (int i = j + 1; i < NP; i++) {
            double t = m[tri(j, i)];
#pragma unroll
            for (int k = 0; k < j; k++) t -= m[tri(k, i)] * m[tri(k, j)];
            m[tri(j, i)] = t / l;
        }
    }
    return true;
}

// Solves L L^T x = b with the factor from cholesky().
__device__ void chol_solve(const double l[28], const double b[NP], double x[NP]) {
    double y[NP];
#pragma unroll
    for (int i = 0; i < NP; i++) {
        double s = b[i];
#pragma unroll
        for (int k = 0; k < i; k++) s -= l[tri(k, i)] * y[k];
        y[i] = s / l[tri(i, i)];
    }
#pragma unroll
    for (int i = NP - 1; i >= 0; i--) {
        double s = y[i];
#pragma unroll
        for (int k = i + 1; k < NP; k++) s -= l[tri(i, k)] * x[k];
        x[i] = s / l[tri(i, i)];
    }
}

// Diagonal of (L L^T)^-1 = L^-T L^-1: entry i is sum_k (L^-1)_{k i}^2.
__device__ void chol_inv_diag(const double l[28], double dg[NP]) {
    double inv[NP][NP];  // lower-triangular L^-1
#pragma unroll
    for (int j = 0; j < NP; j++) {
#pragma unroll
        for (int i = 0; i < NP; i++) {
            if (i < j) {
                inv[i][j] = 0.0;
            } else if (i == j) {
                inv[i][j] = 1.0 / l[tri(i, i)];
            } else {
                double s = 0.0;
#pragma unroll
                for (int k = j; k < i; k++) s -= l[tri(k, i)] * inv[k][j];
                inv[i][j] = s / l[tri(i, i)];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NP; i++) {
        double s = 0.0;
#pragma unroll
        for (int k = i; k < NP; k++) s += inv[k][i] * inv[k][i];
        dg[i] = s;
    }
}

// FWHM along the principal axes of Q and the position angle of the major axis (from +x towards
// +y, in [0, pi)); NaN when Q is not positive definite.
__device__ void gauss_shape(double a, double b, double c, double &maj, double &mnr, double &pa) {
    const double tr = a + c, det = a * c - b * b;
    const double disc = sqrt(fmax(0.0, 0.25 * (a - c) * (a - c) + b * b));
    const double ls = 0.5 * tr - disc, lb = 0.5 * tr + disc;
    if (!(ls > 0.0) || !(det > 0.0)) {
        maj = mnr = pa = NAN;
        return;
    }
    double vx, vy;
    if (fabs(b) + fabs(ls - a) >= fabs(ls - c) + fabs(b)) {
        vx = b;
        vy = ls - a;
    } else {
        vx = ls - c;
        vy = b;
    }
    double t = atan2(vy, vx);
    t = fmod(t, M_PI);
    if (t < 0.0) t += M_PI;
    pa = t;
    maj = FWHM_PER_SIGMA / sqrt(ls);
    mnr = FWHM_PER_SIGMA / sqrt(lb);
}

struct FitArgs {
    const float *img;            // [n_chan][n_pix][n_pix]
    int n_chan, n_pix, half;
    const nbsi_cand *cands;      // null: candidate k is the image centre of channel k (beam fits)
    int n;
    const double *beam;          // [n_chan][3] (FWHM major, minor, angle) or null
    const float2 *stats;         // per channel (median, 1.4826 MAD) or null
    const double *noise_bounds;  // accepted noise range [lo, hi] or null
    double ext_factor;
    nbsi_fit *out;               // [n] or null
    double *beam_out;            // [n][3] or null
};

__global__ __launch_bounds__(64 * S2_WAVES) void gauss_fit_kernel(FitArgs A) {
    __shared__ float s_cut[S2_WAVES][128];
    __shared__ double s_med[S2_WAVES][2];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int k = blockIdx.x * S2_WAVES + wave;
    if (k >= A.n) return;  // the whole wave leaves together
    const int h = A.half, w = 2 * h + 1, npx = w * w, n_pix = A.n_pix;
    int x, y, c;
    if (A.cands) {
        const nbsi_cand cd = A.cands[k];
        x = cd.x;
        y = cd.y;
        c = cd.c;
    } else {
        x = y = n_pix / 2;
        c = k;
    }
    nbsi_fit f;
    f.amp = f.x0 = f.y0 = f.a = f.b = f.c = f.bkg = NAN;
    for (int i = 0; i < NP; i++) f.err[i] = NAN;
    f.fwhm_maj = f.fwhm_min = f.pa = f.rss = f.chi2_red = NAN;
    f.flags = 0;
    f.n_iter = 0;

    const bool chan_ok = c >= 0 && c < A.n_chan;
    double sig = NAN;
    if (chan_ok && A.stats) {
        sig = (double)A.stats[c].y;
        if (A.noise_bounds && !(A.noise_bounds[0] <= sig && sig <= A.noise_bounds[1])) f.flags |= NBSI_S2_NOISY;
    }
    if (!chan_ok || x < h || y < h || x + h >= n_pix || y + h >= n_pix) {
        f.flags = chan_ok ? (f.flags | NBSI_S2_OUTSIDE) : NBSI_S2_OUTSIDE;
        if (lane == 0) {
            if (A.out) A.out[k] = f;
            if (A.beam_out) A.beam_out[3 * k] = A.beam_out[3 * k + 1] = A.beam_out[3 * k + 2] = NAN;
        }
        return;
    }
    double bmaj = NAN, bmin = NAN;
    if (A.beam) {
        bmaj = A.beam[3 * c];
        bmin = A.beam[3 * c + 1];
    }
    const double sigma0 = (isfinite(bmaj) && bmaj > 0.0) ? bmaj / FWHM_PER_SIGMA : 1.0;

    // the lane's pixels: cutout index i = lane and lane + 64, at offsets (i % w - h, i / w - h)
    const float *im = A.img + (size_t)c * n_pix * n_pix;
    double px[2], py[2], d[2];
    bool on[2];
#pragma unroll
    for (int s = 0; s < 2; s++) {
        const int i = lane + 64 * s;
        on[s] = i < npx;
        const int xr = on[s] ? i % w - h : 0, yr = on[s] ? i / w - h : 0;
        px[s] = xr;
        py[s] = yr;
        const float v = on[s] ? im[(size_t)(y + yr) * n_pix + (x + xr)] : 0.0f;
        d[s] = v;
        if (on[s]) s_cut[wave][i] = v;
    }
    // LDS rows are private to the wave (waves of a workgroup may have returned already, so there
    // is no workgroup barrier): the wave's own LDS writes are ordered before other lanes read them
    wave_sync();

    // initial background: median of the 8h border pixels (mean of the two central order
    // statistics), ranks made unique by index
    const int m = 8 * h;
    auto ring = [&](int i) { const int xr = i % w, yr = i / w; return xr == 0 || yr == 0 || xr == w - 1 || yr == w - 1; };
#pragma unroll
    for (int s = 0; s < 2; s++) {
        const int i = lane + 64 * s;
        if (i < npx && ring(i)) {
            const float v = s_cut[wave][i];
            int rank = 0;
            for (int j = 0; j < npx; j++) {
                if (!ring(j)) continue;
                const float u = s_cut[wave][j];
                rank += (u < v || (u == v && j < i)) ? 1 : 0;
            }
            if (rank == (m - 1) / 2) s_med[wave][0] = v;
            if (rank == m / 2) s_med[wave][1] = v;
        }
    }
    wave_sync();
    const double B0 = 0.5 * (s_med[wave][0] + s_med[wave][1]);
    const double dc = (double)s_cut[wave][(npx - 1) / 2];

    double p[NP] = {dc - B0, 0.0, 0.0, 1.0 / (sigma0 * sigma0), 0.0, 1.0 / (sigma0 * sigma0), B0};
    Normal cur, nxt;
    normal_eq(p, px, py, d, on, cur);
    // Levenberg-Marquardt with damping lambda * D, D = the largest diagonal of J^T J seen so far
    // (scale invariant, as in MINPACK), and the gain-ratio update of the damping of Nielsen
    // (Madsen, Nielsen & Tingleff, "Methods for non-linear least squares problems", 2004).
    double D[NP];
#pragma unroll
    for (int i = 0; i < NP; i++) D[i] = 0.0;
    double lambda = 1e-3, nu = 2.0;
    int it = 0;
    for (; it < LM_MAX_IT; it++) {
        double mm[28];
#pragma unroll
        for (int q = 0; q < 28; q++) mm[q] = cur.h[q];
#pragma unroll
        for (int i = 0; i < NP; i++) {
            D[i] = fmax(D[i], cur.h[tri(i, i)]);
            mm[tri(i, i)] += lambda * D[i];
        }
        if (!cholesky(mm)) {
            lambda *= nu;
            nu *= 2.0;
            if (lambda > 1e30) break;
            continue;
        }
        double neg[NP], dl[NP], pn[NP];
#pragma unroll
        for (int i = 0; i < NP; i++) neg[i] = -cur.g[i];
        chol_solve(mm, neg, dl);
        // predicted decrease of the RSS by the linear model: dl . (-2 g - H dl)
        double pred = 0.0;
        bool small = true;
#pragma unroll
        for (int i = 0; i < NP; i++) {
            double hd = 0.0;
#pragma unroll
            for (int j = 0; j < NP; j++) hd += cur.h[i <= j ? tri(i, j) : tri(j, i)] * dl[j];
            pred += dl[i] * (-2.0 * cur.g[i] - hd);
            pn[i] = p[i] + dl[i];
            small = small && fabs(dl[i]) <= 1e-15 * (fabs(p[i]) + 1e-15);
        }
        normal_eq(pn, px, py, d, on, nxt);
        if (isfinite(nxt.rss) && nxt.rss < cur.rss) {
            const double rho = pred > 0.0 ? (cur.rss - nxt.rss) / pred : 0.0;
            const double t = 2.0 * rho - 1.0;
#pragma unroll
            for (int i = 0; i < NP; i++) p[i] = pn[i];
            cur = nxt;
            lambda *= fmax(1.0 / 3.0, 1.0 - t * t * t);
            nu = 2.0;
            if (small) break;
        } else {
            lambda *= nu;
            nu *= 2.0;
            if (lambda > 1e30 || small) break;
        }
    }
    f.n_iter = it;

    bool ok = p[0] > 0.0 && p[3] > 0.0 && p[5] > 0.0 && p[3] * p[5] - p[4] * p[4] > 0.0;
#pragma unroll
    for (int i = 0; i < NP; i++) ok = ok && isfinite(p[i]);
    const int dof = npx - NP;
    if (ok) {
        double l[28];
#pragma unroll
        for (int q = 0; q < 28; q++) l[q] = cur.h[q];
        if (cholesky(l)) {
            double dg[NP];
            chol_inv_diag(l, dg);
#pragma unroll
            for (int i = 0; i < NP; i++) f.err[i] = sqrt(fmax(dg[i] * cur.rss / dof, 0.0));
        } else {
            ok = false;
        }
    }
    f.amp = p[0];
    f.x0 = x + p[1];
    f.y0 = y + p[2];
    f.a = p[3];
    f.b = p[4];
    f.c = p[5];
    f.bkg = p[6];
    f.rss = cur.rss;
    f.chi2_red = (sig > 0.0) ? cur.rss / (sig * sig * dof) : INFINITY;
    if (ok) {
        gauss_shape(p[3], p[4], p[5], f.fwhm_maj, f.fwhm_min, f.pa);
        if (f.fwhm_maj > A.ext_factor * bmaj || f.fwhm_min > A.ext_factor * bmin) f.flags |= NBSI_S2_EXTENDED;
    } else {
        f.flags |= NBSI_S2_FIT_FAILED;
    }
    if (lane == 0) {
        if (A.out) A.out[k] = f;
        if (A.beam_out) {
            A.beam_out[3 * k] = f.fwhm_maj;
            A.beam_out[3 * k + 1] = f.fwhm_min;
            A.beam_out[3 * k + 2] = f.pa;
        }
    }
}

// Accepted range of the channel noise: [med / k, k med] with med the median (mean of the two
// central order statistics) of stats[c].y over the channels.  One workgroup sorts the values in
// LDS (bitonic, padded with +inf to a power of two).
__global__ __launch_bounds__(1024) void noise_bounds_kernel(const float2 *__restrict__ stats, int n_chan, int n_pow2,
                                                            double k, double *__restrict__ bounds) {
    extern __shared__ float s_v[];
    for (int i = threadIdx.x; i < n_pow2; i += blockDim.x) s_v[i] = i < n_chan ? stats[i].y : INFINITY;
    __syncthreads();
    for (int size = 2; size <= n_pow2; size <<= 1) {
        for (int j = size >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n_pow2; i += blockDim.x) {
                const int q = i ^ j;
                if (q > i) {
                    const float a = s_v[i], b = s_v[q];
                    const bool up = (i & size) == 0;
                    if ((a > b) == up) {
                        s_v[i] = b;
                        s_v[q] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        const double med = 0.5 * ((double)s_v[(n_chan - 1) / 2] + (double)s_v[n_chan / 2]);
        bounds[0] = med / k;
        bounds[1] = med * k;
    }
}

__global__ void fill_ones_kernel(float2 *__restrict__ v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        v[i] = make_float2(1.0f, 0.0f);
}

hipError_t launch_fit(const FitArgs &a, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gauss_fit_kernel, dim3((unsigned)((a.n + S2_WAVES - 1) / S2_WAVES)), dim3(64 * S2_WAVES), 0,
                       st, a);
    return hipGetLastError();
}

}  // namespace

extern "C" int nbsi_beam(nbsi_ctx *ctx, const nbsi_image_plan *plan, double *beam) {
    if (!ctx) return NBSI_EINVAL;
    if (!plan || !beam) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_beam: null pointer");
    if (plan->device != ctx->device) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_beam: plan built on another device");
    if (((uintptr_t)beam & 7u) != 0) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_beam: misaligned pointer");
    const int n_pix = plan->n_pix;
    if (n_pix < 2 * NBSI_BEAM_HALF + 2) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_beam: image too small");
    DeviceGuard g(ctx->device);
    const size_t img_chan = (size_t)n_pix * n_pix * sizeof(float);
    const size_t per_chan = (size_t)n_pix * n_pix * sizeof(float2);
    FitArgs fa{};
    fa.n_pix = n_pix;
    fa.half = NBSI_BEAM_HALF;
    fa.ext_factor = INFINITY;
    int rc;
    if (plan->method == NBSI_IMAGE_DFT) {
        // direct Fourier plans: unit float32 visibilities on every product, all channels at once
        const size_t nprod = (size_t)(2 * plan->n_ant) * (2 * plan->n_ant + 1) / 2;
        const size_t vis_bytes = ((nprod * plan->n_chan * sizeof(float2)) + 255) & ~(size_t)255;
        void *buf = nullptr;
        if ((rc = nbsi_scratch(ctx, SLOT_S2_PSF, vis_bytes + img_chan * plan->n_chan, &buf))) return rc;
        float2 *ones = (float2 *)buf;
        float *psf = (float *)((char *)buf + vis_bytes);
        hipLaunchKernelGGL(fill_ones_kernel, dim3(1024), dim3(256), 0, ctx->stream, ones, nprod * plan->n_chan);
        NBSI_TRY_HIP(ctx, hipGetLastError());
        NBSI_TRY_HIP(ctx, launch_image_dft(plan, ones, NBSI_VIS_F32, psf, ctx->stream));
        fa.img = psf;
        fa.n_chan = fa.n = plan->n_chan;
        fa.beam_out = beam;
        NBSI_TRY_HIP(ctx, launch_fit(fa, ctx->stream));
        return NBSI_OK;
    }
    // gridding plans: unit Stokes I on every candidate pair (the gridder keeps those in B), in the
    // imager's channel chunks
    const int chunk = (int)std::max<size_t>(1, std::min<size_t>(plan->n_chan, IMAGE_CHUNK_BYTES / per_chan));
    const size_t ones_n = (size_t)chunk * std::max(1, plan->n_pairs);
    const size_t ones_bytes = (ones_n * sizeof(float2) + 255) & ~(size_t)255;
    void *buf = nullptr, *inter = nullptr;
    if ((rc = nbsi_scratch(ctx, SLOT_S2_PSF, ones_bytes + img_chan * chunk, &buf))) return rc;
    if ((rc = nbsi_scratch(ctx, SLOT_IMG_INTER, per_chan * chunk, &inter))) return rc;
    float2 *ones = (float2 *)buf;
    float *psf = (float *)((char *)buf + ones_bytes);
    hipLaunchKernelGGL(fill_ones_kernel, dim3(1024), dim3(256), 0, ctx->stream, ones, ones_n);
    NBSI_TRY_HIP(ctx, hipGetLastError());
    for (int c0 = 0; c0 < plan->n_chan; c0 += chunk) {
        nbsi_image_plan sub = *plan;
        sub.n_chan = std::min(chunk, plan->n_chan - c0);
        sub.d_freq = plan->d_freq + c0;
        sub.d_nb = plan->d_nb + c0;
        if (plan->d_inb) sub.d_inb = plan->d_inb + (size_t)c0 * ((plan->n_pairs + 31) >> 5);
        NBSI_TRY_HIP(ctx, launch_image_grid_stokes(&sub, ones, NBSI_PREC_FP32, (float2 *)inter, psf, ctx->stream));
        fa.img = psf;
        fa.n_chan = fa.n = sub.n_chan;
        fa.beam_out = beam + 3 * (size_t)c0;
        NBSI_TRY_HIP(ctx, launch_fit(fa, ctx->stream));
    }
    return NBSI_OK;
}

extern "C" int nbsi_stage2(nbsi_ctx *ctx, const float *img, int n_chan, int n_pix, const nbsi_cand *cands,
                           int n_cand, const double *beam, int half, double ext_factor, double noise_k,
                           nbsi_fit *out) {
    if (!ctx) return NBSI_EINVAL;
    if (nbsi_check_detect(n_chan, n_pix, NBSI_DETECT_PER_IMAGE, 0)) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_stage2: bad shape");
    if (n_cand < 0 || n_cand > NBSI_S2_MAX_CANDS) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_stage2: n_cand out of range");
    if (half < 2 || half > NBSI_S2_MAX_HALF) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_stage2: half out of range");
    if (!(ext_factor > 0.0) || !(noise_k >= 1.0)) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_stage2: bad factor");
    if (!img || !beam || (n_cand > 0 && (!cands || !out))) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_stage2: null pointer");
    if (!aligned16(img) || ((uintptr_t)beam & 7u) || ((uintptr_t)cands & 3u) || ((uintptr_t)out & 7u))
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_stage2: misaligned pointer");
    if (n_cand == 0) return NBSI_OK;
    DeviceGuard g(ctx->device);
    void *st = nullptr;
    int rc;
    // per-channel (median, sigma) followed by the two noise bounds
    const size_t stats_bytes = ((size_t)n_chan * sizeof(float2) + 15) & ~(size_t)15;
    if ((rc = nbsi_scratch(ctx, SLOT_DET_STATS, stats_bytes + 2 * sizeof(double), &st))) return rc;
    float *stats = (float *)st;
    double *bounds = (double *)((char *)st + stats_bytes);
    NBSI_TRY_HIP(ctx, launch_detect_stats(img, n_chan, n_pix, NBSI_DETECT_PER_IMAGE, stats, ctx->stream));
    int n_pow2 = 1;
    while (n_pow2 < n_chan) n_pow2 <<= 1;
    const size_t lds = sizeof(float) * (size_t)n_pow2;
    NBSI_TRY_HIP(ctx, hipFuncSetAttribute((const void *)noise_bounds_kernel,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(noise_bounds_kernel, dim3(1), dim3(1024), lds, ctx->stream, (const float2 *)stats, n_chan,
                       n_pow2, noise_k, bounds);
    NBSI_TRY_HIP(ctx, hipGetLastError());
    FitArgs fa{};
    fa.img = img;
    fa.n_chan = n_chan;
    fa.n_pix = n_pix;
    fa.half = half;
    fa.cands = cands;
    fa.n = n_cand;
    fa.beam = beam;
    fa.stats = (const float2 *)stats;
    fa.noise_bounds = bounds;
    fa.ext_factor = ext_factor;
    fa.out = out;
    NBSI_TRY_HIP(ctx, launch_fit(fa, ctx->stream));
    return NBSI_OK;
}
