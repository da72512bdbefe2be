/*
 * Plain CPU oracle for the narrowband spectral-imaging hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or calls this
 * file; only the tests, the smoke check and the benchmark's CPU-baseline leg do.  It shares
 * no code, header, table or constant generator with the HIP path.
 *
 * Everything is FP64 (floating point) or int64 (integer), written for a reader to check
 * against the paper by eye, with no blocking, fusion or reordering beyond the definitions.
 *
 *  - Upchannelisation (Sec. 2.1): an FFT over the time samples of each coarse channel.
 *    A periodic Hann window is applied first, spectra are consecutive non-overlapping
 *    blocks of n_fft samples, no 1/N scaling; fine channel c holds bin k = (c + N/2) mod N.
 *    The FFT is an iterative radix-2 Cooley-Tukey; orc_dft is the O(N^2) definition.
 *  - Requantisation: q = clamp(round-half-even(g * X), -127, 127) per component.
 *  - Cross-correlation (Sec. 2.1): V_ij = sum_s q_i,s conj(q_j,s) for i >= j, accumulated
 *    in int64 and stored in a packed lower triangle t(i,j) = i(i+1)/2 + j.
 *  - Imaging (Sec. 2.2): Stokes I of each antenna pair a > b, (V_XX + V_YY)/2, baseline
 *    (u, v) = (x_a - x_b, y_a - y_b) * nu / c, and the direct Fourier sum
 *    I(l, m) = (1/|B|) sum_b Re[V_b exp(-2 pi i (u l + v m))] on the orthographic grid
 *    l = (x - N/2) * 2/N, m = (y - N/2) * 2/N.
 *
 * Parity pins live in the tests (closed forms, brute force, invariants).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_C_LIGHT 299792458.0
#define ORC_TWO_PI 6.283185307179586476925286766559

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static int is_pow2(long n) { return n > 0 && (n & (n - 1)) == 0; }

/* exp(-2 pi i j / n) with the integer j reduced mod n first, so the angle is exact to rounding. */
static double complex unit_root(long j, long n) {
    long r = j % n;
    if (r < 0) r += n;
    double ang = -ORC_TWO_PI * (double)r / (double)n;
    return cos(ang) + I * sin(ang);
}

/* In-place forward FFT, X[k] = sum_n x[n] exp(-2 pi i k n / N), N a power of two.
 * Iterative radix-2 decimation in time: bit-reversal permutation, then log2 N butterfly stages. */
int orc_fft(double complex *x, long n) {
    if (!is_pow2(n)) return -1;
    for (long i = 1, j = 0; i < n; i++) {
        long bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double complex t = x[i];
            x[i] = x[j];
            x[j] = t;
        }
    }
    for (long len = 2; len <= n; len <<= 1) {
        long half = len >> 1;
        for (long start = 0; start < n; start += len) {
            for (long k = 0; k < half; k++) {
                double complex w = unit_root(k, len);
                double complex a = x[start + k];
                double complex b = x[start + k + half] * w;
                x[start + k] = a + b;
                x[start + k + half] = a - b;
            }
        }
    }
    return 0;
}

/* The definition itself: X[k] = sum_n x[n] exp(-2 pi i k n / N), O(N^2). */
int orc_dft(const double *x_ri, double *X_ri, long n) {
    const double complex *x = (const double complex *)x_ri;
    double complex *X = (double complex *)X_ri;
    for (long k = 0; k < n; k++) {
        double complex acc = 0;
        for (long m = 0; m < n; m++) acc += x[m] * unit_root(k * m, n);
        X[k] = acc;
    }
    return 0;
}

/* FFT of an interleaved (re, im) double array, for tests. */
int orc_fft_ri(double *x_ri, long n) { return orc_fft((double complex *)x_ri, n); }

/* Periodic (DFT-even) Hann window w[n] = 1/2 - 1/2 cos(2 pi n / N). */
double orc_hann(long n, long N) { return 0.5 - 0.5 * cos(ORC_TWO_PI * (double)n / (double)N); }

/*
 * Upchannelise: volt [n_in][n_spec * n_fft][2] int8 -> out [n_chan][n_in][n_spec][2] double,
 * channels chan0 .. chan0 + n_chan - 1 of the fftshifted spectrum.
 */
int orc_channelize(const int8_t *volt, int n_in, int n_fft, int n_spec, int chan0, int n_chan,
                   double *out) {
    if (!is_pow2(n_fft) || n_in <= 0 || n_spec <= 0 || n_chan <= 0) return -1;
    if (chan0 < 0 || chan0 + n_chan > n_fft) return -1;
    const long N = n_fft;
    int err = 0;
#pragma omp parallel
    {
        double complex *buf = (double complex *)malloc(sizeof(double complex) * N);
        if (!buf) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for collapse(2) schedule(dynamic)
        for (int i = 0; i < n_in; i++) {
            for (int s = 0; s < n_spec; s++) {
                if (!buf) continue;
                const int8_t *x = volt + ((long)i * n_spec * N + (long)s * N) * 2;
                for (long n = 0; n < N; n++) {
                    double w = orc_hann(n, N);
                    buf[n] = w * (double)x[2 * n] + I * (w * (double)x[2 * n + 1]);
                }
                orc_fft(buf, N);
                for (int c = chan0; c < chan0 + n_chan; c++) {
                    long k = ((long)c + N / 2) % N;
                    double *o = out + ((((long)(c - chan0) * n_in + i) * n_spec) + s) * 2;
                    o[0] = creal(buf[k]);
                    o[1] = cimag(buf[k]);
                }
            }
        }
        free(buf);
    }
    return err;
}

/*
 * Requantise one component: the decision is taken in float32, the precision of the
 * channelizer arithmetic: p = fl32(fl32(X) * g), q = clamp(round-half-even(p), -127, 127).
 */
static int8_t requant_one(double X, float g) {
    float x32 = (float)X;
    volatile float p = x32 * g;
    float r = nearbyintf(p); /* default rounding mode: to nearest, ties to even */
    if (r > 127.0f) r = 127.0f;
    if (r < -127.0f) r = -127.0f;
    return (int8_t)r;
}

/* spec [n_chan][n_in][n_spec][2] double -> q [n_chan][n_in][2][n_spec] int8 (correlator layout). */
int orc_requantize(const double *spec, int n_chan, int n_in, int n_spec, const float *gain,
                   int8_t *q) {
    for (int c = 0; c < n_chan; c++)
        for (int i = 0; i < n_in; i++)
            for (int s = 0; s < n_spec; s++)
                for (int comp = 0; comp < 2; comp++) {
                    double X = spec[(((long)c * n_in + i) * n_spec + s) * 2 + comp];
                    q[(((long)c * n_in + i) * 2 + comp) * n_spec + s] = requant_one(X, gain[i]);
                }
    return 0;
}

/*
 * Full cross-correlation per channel: V_ij = sum_s q_i,s conj(q_j,s), i >= j (autos included).
 * q: [n_chan][n_in][2][n_spec] int8 (re row, im row).  vis: [n_chan][n_in(n_in+1)/2][2] int32.
 * Returns -3 if any accumulated value does not fit in int32.
 */
int orc_correlate(const int8_t *q, int n_chan, int n_in, int n_spec, int32_t *vis) {
    const long nprod = (long)n_in * (n_in + 1) / 2;
    int overflow = 0;
#pragma omp parallel for schedule(dynamic) reduction(| : overflow)
    for (int c = 0; c < n_chan; c++) {
        const int8_t *qc = q + (long)c * n_in * 2 * n_spec;
        for (int i = 0; i < n_in; i++) {
            const int8_t *ar = qc + (long)i * 2 * n_spec, *ai = ar + n_spec;
            for (int j = 0; j <= i; j++) {
                const int8_t *br = qc + (long)j * 2 * n_spec, *bi = br + n_spec;
                int64_t re = 0, im = 0;
                for (int s = 0; s < n_spec; s++) {
                    /* (ar + i ai)(br - i bi) = (ar br + ai bi) + i (ai br - ar bi) */
                    re += (int64_t)ar[s] * br[s] + (int64_t)ai[s] * bi[s];
                    im += (int64_t)ai[s] * br[s] - (int64_t)ar[s] * bi[s];
                }
                if (re > INT32_MAX || re < INT32_MIN || im > INT32_MAX || im < INT32_MIN)
                    overflow = 1;
                long t = (long)i * (i + 1) / 2 + j;
                vis[((long)c * nprod + t) * 2] = (int32_t)re;
                vis[((long)c * nprod + t) * 2 + 1] = (int32_t)im;
            }
        }
    }
    return overflow ? -3 : 0;
}

/*
 * The imaged baseline set B for one channel.  A pair a > b is kept when
 *   uv_min <= sqrt(u^2 + v^2) <= uv_max, and, for the gridded method (grid_n_pix > 0),
 *   |u| <= U and |v| <= U with U = (sigma N / 2 - w / 2 - 1) * du, sigma = 2, w = 8,
 *   du = 1 / (2 sigma) wavelengths, so every kernel tap stays inside the oversampled grid.
 * u = ((x_a - x_b) * nu) / c, v likewise; written with explicit operation order.
 */
static int in_set(double u, double v, int grid_n_pix, double uv_min, double uv_max) {
    double r = sqrt(u * u + v * v);
    if (r < uv_min || r > uv_max) return 0;
    if (grid_n_pix > 0) {
        const double sigma = 2.0, w = 8.0, du = 1.0 / (2.0 * sigma);
        double U = (sigma * grid_n_pix / 2.0 - w / 2.0 - 1.0) * du;
        if (fabs(u) > U || fabs(v) > U) return 0;
    }
    return 1;
}

static void baseline_uv(const double *xyz, int a, int b, double nu, double *u, double *v) {
    double dx = xyz[3 * a] - xyz[3 * b];
    double dy = xyz[3 * a + 1] - xyz[3 * b + 1];
    double px = dx * nu, py = dy * nu;
    *u = px / ORC_C_LIGHT;
    *v = py / ORC_C_LIGHT;
}

/* Number of imaged baselines per channel. */
int orc_count_baselines(int n_chan, int n_ant, const double *xyz, const double *freq,
                        int grid_n_pix, double uv_min, double uv_max, int64_t *n_b) {
    for (int c = 0; c < n_chan; c++) {
        int64_t cnt = 0;
        for (int a = 0; a < n_ant; a++)
            for (int b = 0; b < a; b++) {
                double u, v;
                baseline_uv(xyz, a, b, freq[c], &u, &v);
                cnt += in_set(u, v, grid_n_pix, uv_min, uv_max);
            }
        n_b[c] = cnt;
    }
    return 0;
}

/*
 * Direct Fourier imager.  vis: [n_chan][n_in(n_in+1)/2][2] double (n_in = 2 n_ant), img:
 * [n_chan][n_pix][n_pix] double with row y <-> m, column x <-> l.  The phase is formed in
 * turns, reduced to its fractional part, then cos/sin of 2 pi * frac.  Channels with an empty
 * set B give an all-zero image.
 */
int orc_image_dft(const double *vis, int n_chan, int n_ant, const double *xyz, const double *freq,
                  int n_pix, int grid_n_pix, double uv_min, double uv_max, double *img) {
    const int n_in = 2 * n_ant;
    const long nprod = (long)n_in * (n_in + 1) / 2;
    const long nbl = (long)n_ant * (n_ant - 1) / 2;
    double *bu = (double *)malloc(sizeof(double) * nbl);
    double *bv = (double *)malloc(sizeof(double) * nbl);
    double *vr = (double *)malloc(sizeof(double) * nbl);
    double *vi = (double *)malloc(sizeof(double) * nbl);
    if (!bu || !bv || !vr || !vi) {
        free(bu); free(bv); free(vr); free(vi);
        return -2;
    }
    for (int c = 0; c < n_chan; c++) {
        const double *vc = vis + (long)c * nprod * 2;
        long nb = 0;
        for (int a = 0; a < n_ant; a++)
            for (int b = 0; b < a; b++) {
                double u, v;
                baseline_uv(xyz, a, b, freq[c], &u, &v);
                if (!in_set(u, v, grid_n_pix, uv_min, uv_max)) continue;
                long txx = (long)(2 * a) * (2 * a + 1) / 2 + 2 * b;
                long tyy = (long)(2 * a + 1) * (2 * a + 2) / 2 + 2 * b + 1;
                bu[nb] = u;
                bv[nb] = v;
                vr[nb] = 0.5 * (vc[2 * txx] + vc[2 * tyy]);
                vi[nb] = 0.5 * (vc[2 * txx + 1] + vc[2 * tyy + 1]);
                nb++;
            }
        double *ic = img + (long)c * n_pix * n_pix;
#pragma omp parallel for collapse(2) schedule(static)
        for (int y = 0; y < n_pix; y++)
            for (int x = 0; x < n_pix; x++) {
                double l = (x - n_pix / 2) * (2.0 / n_pix);
                double m = (y - n_pix / 2) * (2.0 / n_pix);
                double acc = 0.0;
                for (long b = 0; b < nb; b++) {
                    double turns = bu[b] * l + bv[b] * m;
                    double frac = turns - floor(turns);
                    double th = ORC_TWO_PI * frac;
                    /* Re[(vr + i vi) (cos th - i sin th)] */
                    acc += vr[b] * cos(th) + vi[b] * sin(th);
                }
                ic[(long)y * n_pix + x] = nb > 0 ? acc / (double)nb : 0.0;
            }
    }
    free(bu); free(bv); free(vr); free(vi);
    return 0;
}

/*
 * The same direct Fourier sum evaluated only at a list of pixels (x, y) (for spot checks of
 * large images): out [n_chan][n_list].
 */
int orc_image_dft_pixels(const double *vis, int n_chan, int n_ant, const double *xyz,
                         const double *freq, int n_pix, int grid_n_pix, double uv_min,
                         double uv_max, const int32_t *pix_xy, int n_list, double *out) {
    const int n_in = 2 * n_ant;
    const long nprod = (long)n_in * (n_in + 1) / 2;
    const long nbl = (long)n_ant * (n_ant - 1) / 2;
    int err = 0;
#pragma omp parallel for schedule(dynamic)
    for (int c = 0; c < n_chan; c++) {
        double *bu = (double *)malloc(sizeof(double) * nbl);
        double *bv = (double *)malloc(sizeof(double) * nbl);
        double *vr = (double *)malloc(sizeof(double) * nbl);
        double *vi = (double *)malloc(sizeof(double) * nbl);
        if (!bu || !bv || !vr || !vi) {
            free(bu); free(bv); free(vr); free(vi);
#pragma omp atomic write
            err = -2;
            continue;
        }
        const double *vc = vis + (long)c * nprod * 2;
        long nb = 0;
        for (int a = 0; a < n_ant; a++)
            for (int b = 0; b < a; b++) {
                double u, v;
                baseline_uv(xyz, a, b, freq[c], &u, &v);
                if (!in_set(u, v, grid_n_pix, uv_min, uv_max)) continue;
                long txx = (long)(2 * a) * (2 * a + 1) / 2 + 2 * b;
                long tyy = (long)(2 * a + 1) * (2 * a + 2) / 2 + 2 * b + 1;
                bu[nb] = u;
                bv[nb] = v;
                vr[nb] = 0.5 * (vc[2 * txx] + vc[2 * tyy]);
                vi[nb] = 0.5 * (vc[2 * txx + 1] + vc[2 * tyy + 1]);
                nb++;
            }
        for (int q = 0; q < n_list; q++) {
            int x = pix_xy[2 * q], y = pix_xy[2 * q + 1];
            double l = (x - n_pix / 2) * (2.0 / n_pix);
            double m = (y - n_pix / 2) * (2.0 / n_pix);
            double acc = 0.0;
            for (long b = 0; b < nb; b++) {
                double turns = bu[b] * l + bv[b] * m;
                double frac = turns - floor(turns);
                double th = ORC_TWO_PI * frac;
                acc += vr[b] * cos(th) + vi[b] * sin(th);
            }
            out[(long)c * n_list + q] = nb > 0 ? acc / (double)nb : 0.0;
        }
        free(bu); free(bv); free(vr); free(vi);
    }
    return err;
}
