/*
 * nbsi.h - C ABI of the MI355X (gfx950) narrowband spectral-imaging library.
 *
 * The calls follow the paper's statement of the problem (arXiv 2606.04304, Sec. 2.1-2.4):
 * upchannelise coarse-channel voltages, cross-correlate every baseline per fine channel,
 * image every fine channel over the visible hemisphere, and search the spectral cube for
 * narrowband outliers.
 *
 * Conventions shared by every call
 *  - Array arguments are DEVICE pointers unless the name ends in _host.  The caller owns all
 *    buffers; the library never frees or keeps them beyond the work it enqueues.
 *  - Every call first validates its arguments on the host.  On a bad argument it returns a
 *    negative status and enqueues nothing.  Otherwise it enqueues its kernels asynchronously
 *    on the context's stream and returns NBSI_OK (nbsi_detect alone blocks, to return the
 *    candidate count).
 *  - Device pointers must be 16-byte aligned.  No C++ exception crosses this interface.
 *  - A context is not thread-safe; use one context per host thread / stream.  Scratch memory
 *    is owned by the context, grown on demand and released by nbsi_destroy.
 *  - Complex numbers are stored as (re, im) pairs.  Input i belongs to antenna i / 2 and
 *    polarisation i % 2 (0 = X, 1 = Y).
 */
#ifndef NBSI_H
#define NBSI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NBSI_OK 0
#define NBSI_EINVAL (-1)       /* bad shape, null or misaligned pointer, bad enum */
#define NBSI_EOVERFLOW (-2)    /* a result could not fit its type (e.g. n_spec > 65535) */
#define NBSI_ENOMEM (-3)       /* scratch allocation failed */
#define NBSI_EHIP (-4)         /* a HIP runtime call failed (detail in nbsi_last_error) */
#define NBSI_ETRUNC (-5)       /* output buffer too short; *n_out holds the true count */
#define NBSI_EUNSUPPORTED (-6) /* valid request this build does not implement */

#define NBSI_MAX_SPEC 65535    /* int32 visibilities are exact up to this many spectra */

/* imaging methods */
#define NBSI_IMAGE_DFT 0       /* direct Fourier sum over every imaged baseline */
#define NBSI_IMAGE_GRID 1      /* ES-kernel gridding on a 2x oversampled grid + 2D FFT */

/* visibility input types of nbsi_image */
#define NBSI_VIS_I32 0
#define NBSI_VIS_F32 1

/* gridding arithmetic of nbsi_image (accumulation is FP32 in every mode) */
#define NBSI_PREC_FP32 0
#define NBSI_PREC_FP16 1
#define NBSI_PREC_BF16 2

/* detector noise models */
#define NBSI_DETECT_PER_PIXEL 0
#define NBSI_DETECT_PER_IMAGE 1

typedef struct nbsi_ctx nbsi_ctx;
typedef struct nbsi_image_plan nbsi_image_plan;

/* One candidate (Sec. 2.4: sky position, detection frequency, effective width, SNR). */
typedef struct {
    int32_t x;      /* pixel column (l) */
    int32_t y;      /* pixel row (m) */
    int32_t c;      /* channel index within the cube */
    int32_t width;  /* matched-filter width in channels */
    float snr;
} nbsi_cand;

int nbsi_version(void);
const char *nbsi_strerror(int status);

/* Create a context on HIP device `device` that enqueues on `stream` (a hipStream_t; NULL =
 * the default stream).  Returns NBSI_EHIP if the device cannot be used. */
int nbsi_create(nbsi_ctx **ctx, int device, void *stream);
int nbsi_destroy(nbsi_ctx *ctx);
/* Enqueue later calls on `stream`.  When it differs from the current one, the new stream first
 * waits for all work the context enqueued before (the context's scratch is shared by its
 * calls, so calls on different streams of one context never overlap). */
int nbsi_set_stream(nbsi_ctx *ctx, void *stream);
/* Human-readable detail of the last failure on this context ("" if none). */
const char *nbsi_last_error(const nbsi_ctx *ctx);
/* Wait for all work enqueued by this context. */
int nbsi_synchronize(nbsi_ctx *ctx);

/*
 * Device-side status of a context: bits that kernels set when they meet non-finite numbers or
 * saturate (the data conditions a caller cannot see from the return codes, which report only
 * argument and runtime errors):
 *   NBSI_FLAG_SPEC_NONFINITE  nbsi_channelize: some g_i X was not finite (a non-finite or
 *                             overflowing gain); its spec_f value is written as computed and
 *                             its int8 code is 0.
 *   NBSI_FLAG_SPEC_CLIPPED    nbsi_channelize: some requantised component saturated at +-127.
 *   NBSI_FLAG_IMAGE_NONFINITE nbsi_image, nbsi_image_stokes, nbsi_correlate_image, nbsi_batch_run:
 *                             some output pixel is not finite (a non-finite input visibility
 *                             in the imaged set, which spreads over the image).
 *   NBSI_FLAG_CUBE_NONFINITE  nbsi_detect, nbsi_detect_noalloc: some pixel inside the visible
 *                             hemisphere has a non-finite value in its spectrum; that pixel is
 *                             not searched (its SNR output is 0, as outside the hemisphere),
 *                             and PER_IMAGE statistics use each channel's finite pixels only.
 * nbsi_status waits for the context's work (its stream and auxiliary stream), stores the bits
 * set since the previous nbsi_status of this context (or its creation) in *flags_host and
 * clears them.  Kernels of every call on the context set them; contexts do not share them.
 */
#define NBSI_FLAG_SPEC_NONFINITE 1
#define NBSI_FLAG_SPEC_CLIPPED 2
#define NBSI_FLAG_IMAGE_NONFINITE 4
#define NBSI_FLAG_CUBE_NONFINITE 8
int nbsi_status(nbsi_ctx *ctx, uint32_t *flags_host);

/*
 * Host-only argument checks, also run first by each call below.  They need no GPU.
 * nbsi_check_channelize: n_fft a power of two in [2^8, 2^18]; 1 <= n_spec <= NBSI_MAX_SPEC;
 *   n_chan >= 1, 0 <= chan0, chan0 + n_chan <= n_fft, n_chan <= 16384 (the kept band must fit
 *   one on-chip sub-transform); n_in >= 1.
 * nbsi_check_correlate: n_in >= 1, n_chan >= 1, 1 <= n_spec <= NBSI_MAX_SPEC.
 * nbsi_check_image: n_ant >= 2, n_chan >= 1, n_pix even in [8, 1024], method and precision
 *   valid, 0 <= uv_min <= uv_max.
 * nbsi_check_detect: n_chan >= 3, n_pix even in [8, 1024], mode valid, max_out >= 0.
 */
int nbsi_check_channelize(int n_in, int n_fft, int n_spec, int chan0, int n_chan);
int nbsi_check_correlate(int n_chan, int n_in, int n_spec);
int nbsi_check_image(int n_chan, int n_ant, int n_pix, int method, int precision,
                     double uv_min, double uv_max);
int nbsi_check_detect(int n_chan, int n_pix, int mode, int max_out);

/*
 * Upchannelisation and requantisation (Sec. 2.1: an FFT over the time samples of each
 * coarse channel raises the spectral resolution; the selected fine channels form a batch).
 *   volt   [n_in][n_spec * n_fft][2] int8: complex voltages, time-contiguous per input.
 *   gain   [n_in] float32: per-input requantisation gain g_i.
 * For input i and spectrum s (samples s*n_fft .. s*n_fft + n_fft - 1):
 *   X[k] = sum_n w[n] x[n] exp(-2 pi i k n / n_fft), w[n] = 1/2 - 1/2 cos(2 pi n / n_fft)
 *   (periodic Hann), no 1/N scaling.  Fine channel c holds bin k = (c + n_fft/2) mod n_fft
 *   (fftshift), and channels chan0 .. chan0 + n_chan - 1 are kept.
 * Outputs (either may be NULL, not both), correlator layout [n_chan][n_in][2][n_spec]
 * (for each channel and input: n_spec real parts, then n_spec imaginary parts):
 *   spec_f float32: g_i * X, computed in float32;
 *   spec_q int8:    clamp(round-half-even(g_i * X), -127, 127), the float32 value of spec_f.
 */
int nbsi_channelize(nbsi_ctx *ctx, const int8_t *volt, int n_in, int n_fft, int n_spec,
                    int chan0, int n_chan, const float *gain, int8_t *spec_q, float *spec_f);

/*
 * Full cross-correlation (Sec. 2.1, the X-engine): for every channel and every pair i >= j,
 *   V_ij = sum_{s < n_spec} q_i,s conj(q_j,s)
 * on int8 matrix cores with int32 accumulation, exact for n_spec <= NBSI_MAX_SPEC (any int8,
 * including -128).
 *   spec_q [n_chan][n_in][2][n_spec] int8 (nbsi_channelize layout).
 *   vis    [n_chan][n_in (n_in + 1) / 2][2] int32, packed lower triangle t(i, j) = i(i+1)/2 + j.
 */
int nbsi_correlate(nbsi_ctx *ctx, const int8_t *spec_q, int n_chan, int n_in, int n_spec,
                   int32_t *vis);

/* Name of the kernel nbsi_correlate runs for this shape (a static string; host only):
 * "correlate_i8_chan_kernel<32>" / "<64>" (short integrations: one workgroup holds a whole
 * channel), "correlate_i8_pipe_kernel<256>" (256 x 256 tiles, integrations of more than 64
 * spectra) or "correlate_i8_pipe_kernel<128>" (128 x 128 tiles: up to 64 spectra of more inputs
 * than the whole-channel kernels hold in LDS). */
const char *nbsi_correlate_kernel(int n_in, int n_spec);

/*
 * Correlation with calibration applied in the epilogue (Sec. 2.2: per-antenna complex gains and
 * bandpass solutions applied before imaging; solving for them is not part of this library):
 *   vis_cal[c][t(i, j)] = w_i[c] * V_ij[c] * conj(w_j[c]),
 * with V_ij the exact int32 sum of nbsi_correlate rounded to float32 and the products formed in
 * float32.  cal [n_chan][n_in][2] float32 (device, 8-byte aligned) holds the complex correction
 * factors (the inverse of the measured gains, bandpass included) of every input and channel;
 * vis_cal [n_chan][n_in (n_in + 1) / 2][2] float32, the nbsi_correlate layout, feeds nbsi_image
 * with NBSI_VIS_F32.  Shapes and errors as nbsi_correlate.
 */
int nbsi_correlate_cal(nbsi_ctx *ctx, const int8_t *spec_q, int n_chan, int n_in, int n_spec,
                       const float *cal, float *vis_cal);

/* The same product from float32 spectra (the plain FP32 path): vis in float32, same layout. */
int nbsi_correlate_f32(nbsi_ctx *ctx, const float *spec_f, int n_chan, int n_in, int n_spec,
                       float *vis);

/*
 * Imaging geometry (Sec. 2.2: all-sky images of every fine channel over the visible
 * hemisphere).  A plan fixes the antennas, the channel frequencies, the image size and the
 * method; it is built on the host, uploaded once, and reused by nbsi_image.
 *   ant_xyz_host [n_ant][3] float64 metres (z is ignored: coplanar array).
 *   freq_hz_host [n_chan] float64 sky frequency of each channel.
 * Baseline a > b has (u, v) = ((x_a - x_b) * nu / c, (y_a - y_b) * nu / c) wavelengths.
 * Imaged set B per channel: pairs with uv_min <= |uv| <= uv_max, and for NBSI_IMAGE_GRID also
 * |u|, |v| <= (2 n_pix / 2 - 4 - 1) / 4 (every tap of the width-8 kernel stays on the 2x grid).
 */
int nbsi_image_plan_create(nbsi_ctx *ctx, const double *ant_xyz_host, int n_ant,
                           const double *freq_hz_host, int n_chan, int n_pix, int method,
                           double uv_min, double uv_max, nbsi_image_plan **plan);
int nbsi_image_plan_destroy(nbsi_image_plan *plan);
/* Copy |B| per channel into n_b_host[n_chan] (blocks until the plan is built). */
int nbsi_image_plan_nbase(nbsi_image_plan *plan, int64_t *n_b_host);

/*
 * Dirty image of every channel (Stokes I, natural weighting):
 *   I(l, m) = (1/|B|) sum_{b in B} Re[V_I,b exp(-2 pi i (u_b l + v_b m))],
 *   V_I = (V_XX + V_YY) / 2 of antennas a > b (autos and cross-hands unused),
 *   l = (x - n_pix/2) * 2/n_pix, m = (y - n_pix/2) * 2/n_pix.
 *   vis  [n_chan][n_in (n_in+1)/2][2] int32 (NBSI_VIS_I32) or float32 (NBSI_VIS_F32),
 *        n_in = 2 n_ant.
 *   img  [n_chan][n_pix][n_pix] float32, row y <-> m, column x <-> l.
 * NBSI_IMAGE_DFT evaluates the sum directly (float64 phases).  NBSI_IMAGE_GRID grids with the
 * exponential-of-semicircle kernel (width 8, beta = 2.30 * 8) onto a 2 n_pix square grid,
 * transforms it with a 2D FFT and divides by the kernel's Fourier transform; `precision`
 * selects the gridding arithmetic (FP32, FP16 or BF16 products, FP32 accumulation) and
 * applies to NBSI_IMAGE_GRID only.  uv coordinates are float64 on the GPU.
 */
int nbsi_image(nbsi_ctx *ctx, const nbsi_image_plan *plan, const void *vis, int vis_dtype,
               int precision, float *img);

/*
 * Correlate and image without re-reading the visibilities (Sec. 2.1 X-engine feeding the
 * Sec. 2.2 imager).  A gridding plan lists its candidate pairs (every pair a > b that is in B
 * for some channel of the plan); nbsi_image_plan_pairs gives their number n_pairs and, if
 * pairs_host is not NULL, copies them as pairs_host[n_pairs][2] = (a, b) (blocking).
 * nbsi_correlate_stokes writes exactly what nbsi_correlate writes to vis and, from the same
 * int32 sums, V_I = (V_XX + V_YY) / 2 of every candidate pair into
 *   stokes_i [n_chan][n_pairs][2] float32 (real, imaginary; rounded from the exact sum),
 * requiring n_in = 2 n_ant and n_chan of the plan.  nbsi_image_stokes images those values
 * (applying the per-channel membership test of B itself) and gives, bit for bit, what
 * nbsi_image gives from vis with the same plan and precision.  Gridding plans only
 * (NBSI_EINVAL otherwise); stokes_i is caller-owned device memory, 16-byte aligned.
 */
int nbsi_image_plan_pairs(const nbsi_image_plan *plan, int *n_pairs_host, int32_t *pairs_host);
int nbsi_correlate_stokes(nbsi_ctx *ctx, const int8_t *spec_q, int n_chan, int n_in, int n_spec,
                          const nbsi_image_plan *plan, int32_t *vis, float *stokes_i);
int nbsi_image_stokes(nbsi_ctx *ctx, const nbsi_image_plan *plan, const float *stokes_i,
                      int precision, float *img);

/*
 * Both of the above with the two stages overlapped (the X-engine and imager of Sec. 2.1 run as
 * a pipeline over channel chunks, as the paper's batches stream through its GPU stages):
 * the channels are cut into n_stages ranges of whole imaging chunks (0 = NBSI_DEFAULT_STAGES,
 * at most NBSI_MAX_STAGES; fewer when the plan has fewer chunks); range k is correlated on the
 * context's stream while range k - 1 is imaged on an auxiliary stream of the context (created
 * on first use, default priority), and the context's stream waits for the last image before
 * its next work.  vis, stokes_i and img receive, bit for bit, what nbsi_correlate_stokes
 * followed by nbsi_image_stokes write; same shapes, alignment and ownership.  Two calls on
 * one context are ordered like any other work of the context; concurrent calls on one
 * context from several host threads race (as for every entry point).
 */
#define NBSI_MAX_STAGES 64
#define NBSI_DEFAULT_STAGES 16
int nbsi_correlate_image(nbsi_ctx *ctx, const int8_t *spec_q, int n_chan, int n_in, int n_spec,
                         const nbsi_image_plan *plan, int precision, int n_stages, int32_t *vis,
                         float *stokes_i, float *img);

/*
 * Narrowband search of a cube (Sec. 2.4, Stage I with the width-1 matched filter):
 *   NBSI_DETECT_PER_PIXEL: SNR_p[c] = (I_p[c] - med_c I_p) / (k MAD_c I_p)
 *   NBSI_DETECT_PER_IMAGE: z = (I - med) / (k MAD) over each channel image, then
 *                          SNR_p[c] = z_p[c] - med_c z_p
 *   with k = 1.482602218505602, the median of an even count the mean of the central pair,
 *   over pixels with (x - n/2)^2 + (y - n/2)^2 < (n/2)^2 (the visible hemisphere).
 * A voxel is a candidate when SNR >= thresh and it has the highest SNR within +-1 channel
 * (non-maximum suppression, ties keep the lower channel).  Pixels with MAD = 0 are skipped.
 *   img     [n_chan][n_pix][n_pix] float32.
 *   snr     optional [n_chan][n_pix][n_pix] float32 SNR cube (0 outside the searched pixels).
 *   out     [max_out] candidates sorted by (y, x, c); n_out (HOST) receives the true count.
 * Returns NBSI_ETRUNC when the count exceeds max_out (the first max_out are written).
 * Blocks until the count is known.
 */
int nbsi_detect(nbsi_ctx *ctx, const float *img, int n_chan, int n_pix, int mode, float thresh,
                float *snr, nbsi_cand *out, int max_out, int *n_out);

/*
 * nbsi_detect for callers that cannot allocate device memory (serving loops, harnesses that
 * forbid hipMalloc): the same kernels and results, with the detector's statistics, candidate
 * buffer, sort keys and counter in a fixed workspace of NBSI_DETECT_NOALLOC_BYTES per GPU
 * (a static device array, resolved by nbsi_create and held until the process ends); the call
 * allocates nothing.  Same arguments, layouts and ownership as nbsi_detect.  More than
 * NBSI_DETECT_NOALLOC_MAX_CANDS candidates (before truncation to max_out) returns
 * NBSI_EOVERFLOW with nothing written to out.  Every call on one GPU shares that GPU's
 * workspace: calls that overlap on one GPU (several contexts or streams at once) race.
 * Blocks until the result is written.
 */
#define NBSI_DETECT_NOALLOC_MAX_CANDS 65536
#define NBSI_DETECT_NOALLOC_BYTES 2097408
int nbsi_detect_noalloc(nbsi_ctx *ctx, const float *img, int n_chan, int n_pix, int mode,
                        float thresh, float *snr, nbsi_cand *out, int max_out, int *n_out);

/*
 * Full Stage I search (Sec. 2.4: matched filtering over line widths, FDR control, suppression of
 * repeated triggers along frequency, local re-evaluation) on a standardised residual cube
 * snr [n_chan][n_pix][n_pix] (e.g. nbsi_detect's PER_PIXEL or PER_IMAGE SNR output):
 *   1. S_w[c] = (1/sqrt(w)) sum_{j<w} snr[c - floor(w/2) + j] for every width w of the bank whose
 *      window lies inside the band; per voxel the largest S and its width (the narrower on ties).
 *      widths_host NULL selects 1..10, 12..48 step 4, 50..100 step 10 (26 widths); otherwise
 *      n_widths in [1, NBSI_SEARCH_MAX_WIDTHS] widths in [1, NBSI_SEARCH_MAX_WIDTH].
 *   2. p = erfc(S / sqrt 2) / 2; Benjamini-Hochberg at level fdr_q in (0, 1) over the
 *      m = (in-horizon pixels) x n_chan voxels: the k* largest S are provisional detections,
 *      k* = max{k : p_(k) <= k fdr_q / m}, exactly, for every fdr_q (BH accepts no
 *      p-value above fdr_q, so only S >= Q^-1(fdr_q) are ranked; values of S are compared in
 *      float32 as the kernel computed them, p in float64 from libm erfc).
 *   3. A provisional detection survives when no other one at its pixel within max(floor(w/2), 1)
 *      channels is higher (a lower channel wins ties), and
 *   4. when its SNR recomputed against the median and 1.4826 MAD of its flanks (guard w,
 *      max(16, 2w) channels each side, at least 8 in all) is >= the BH threshold S* (the k*-th
 *      largest S).
 * out (device, sorted by (y, x, c)) receives {x, y, c, width, snr = S}; *n_out the survivor count
 * (NBSI_ETRUNC if above max_out); thresh_host (optional) S*, +inf when nothing is accepted;
 * n_provisional_host (optional) k*.  best_snr [n_chan][n_pix][n_pix] float32 and best_width
 * (same shape, uint8) are optional device outputs of step 1 (context scratch when NULL).
 * Blocks until the result is on the host.
 */
#define NBSI_SEARCH_MAX_WIDTHS 32
#define NBSI_SEARCH_MAX_WIDTH 128
int nbsi_search(nbsi_ctx *ctx, const float *snr, int n_chan, int n_pix, const int32_t *widths_host,
                int n_widths, double fdr_q, float *best_snr, uint8_t *best_width, nbsi_cand *out,
                int max_out, int *n_out, float *thresh_host, int64_t *n_provisional_host);

/*
 * The Stage I search of nbsi_search on a cube whose noise is correlated across channels (Sec.
 * 2.4's unit-normalised boxcars read as unit variance under that correlation).  rho_host (host,
 * n_rho values, NULL when n_rho = 0) holds the correlation of the cube's noise at lags of
 * 1 .. n_rho channels (zero beyond); every window sum of width w is divided by
 *   sigma_w = sqrt(w + 2 sum_{l=1}^{min(w-1, n_rho)} (w - l) rho_l)
 * in place of sqrt(w), in step 1 and in the re-evaluation of step 4.  The images of this library
 * (periodic Hann window, cross-correlations of independent inputs) have rho = (4/9, 1/36).
 * n_rho in [0, NBSI_SEARCH_MAX_LAG], each rho in (-1, 1), and sigma_w^2 > 0 for every width of
 * the bank, else NBSI_EINVAL.  n_rho = 0 is nbsi_search.  Other arguments, layouts, ownership
 * and errors as nbsi_search.
 */
#define NBSI_SEARCH_MAX_LAG 8
int nbsi_search_corr(nbsi_ctx *ctx, const float *snr, int n_chan, int n_pix, const int32_t *widths_host,
                     int n_widths, const double *rho_host, int n_rho, double fdr_q, float *best_snr,
                     uint8_t *best_width, nbsi_cand *out, int max_out, int *n_out, float *thresh_host,
                     int64_t *n_provisional_host);

/*
 * Drift-rate search (the paper's Doppler-drift discussion, Sec. 2: a search over drifts of tens
 * of Hz per dump): snr_sub [n_sub][n_chan][n_pix][n_pix] float32 holds the standardised residual
 * cubes of n_sub sub-integrations of one dump (each channelised, correlated, imaged and
 * standardised with this library).  For every total drift d = -max_drift..max_drift channels
 * over the dump and every start channel c whose track stays in the band (0 <= c + d < n_chan),
 *   D_d[c] = (1/sqrt(n_sub)) sum_s snr_sub[s][c + shift(d, s)],
 *   shift(d, s) = round(d s / (n_sub - 1)), halves away from zero (0 when n_sub = 1);
 * best [n_chan][n_pix][n_pix] float32 receives max_d D_d (-inf where no track fits) and drift
 * (same shape, int8) its d, trials taken in the order 0, -1, +1, -2, ... (ties keep the first).
 * 1 <= n_sub <= NBSI_DEDOPPLER_MAX_SUB, 0 <= max_drift <= NBSI_DEDOPPLER_MAX_DRIFT; device
 * pointers 16-byte aligned.  Asynchronous on the context's stream.
 */
#define NBSI_DEDOPPLER_MAX_SUB 8
#define NBSI_DEDOPPLER_MAX_DRIFT 16
int nbsi_dedoppler(nbsi_ctx *ctx, const float *snr_sub, int n_sub, int n_chan, int n_pix, int max_drift,
                   float *best, int8_t *drift);

/*
 * Stage II automated cuts (Sec. 2.4: candidates consistent with narrowband point sources are
 * kept; extended morphology is rejected, images with deviant noise are flagged; positions come
 * from Gaussian centroid fits whose covariance errors are rescaled by sqrt(reduced chi-square)).
 *
 * Fit of one cutout: the (2 half + 1)^2 pixels of the candidate's channel image centred on its
 * pixel, model f = bkg + amp exp(-Q/2), Q = a dx^2 + 2 b dx dy + c dy^2 with dx, dy measured from
 * the centroid (x0, y0), least squares with unit weights (Levenberg-Marquardt in FP64, started
 * from amp = centre - bkg, the pixel itself, a = c = 1/sigma^2 with sigma = the beam's major
 * FWHM / 2 sqrt(2 ln 2), or 1 pixel without a beam, b = 0, bkg = median of the border pixels).
 * err[i] = sqrt(((J^T J)^-1)_ii RSS / (n - 7)), n the pixel count; chi2_red = RSS / (sigma_c^2
 * (n - 7)) with sigma_c the channel image's 1.4826 MAD over the visible hemisphere.  FWHM of the
 * principal axes 2 sqrt(2 ln 2) / sqrt(eigenvalue of [[a, b], [b, c]]) in pixels; pa: angle of
 * the major axis from +x towards +y, radians in [0, pi).
 */
#define NBSI_S2_FIT_FAILED 1 /* amp <= 0, Q not positive definite, or singular normal matrix */
#define NBSI_S2_EXTENDED 2   /* major or minor FWHM above ext_factor times the beam's */
#define NBSI_S2_NOISY 4      /* sigma_c outside [m / noise_k, noise_k m], m = median of sigma_c */
#define NBSI_S2_OUTSIDE 8    /* cutout not inside the image, or channel outside the cube */
#define NBSI_S2_MAX_HALF 5
#define NBSI_S2_MAX_CANDS (1 << 22)
#define NBSI_BEAM_HALF 2
typedef struct {
    double amp, x0, y0, a, b, c, bkg; /* x0, y0 in image pixels (x = column, y = row) */
    double err[7];                    /* 1-sigma errors, same order */
    double fwhm_maj, fwhm_min, pa;
    double rss, chi2_red;
    int32_t flags; /* NBSI_S2_* bits; 0 = kept */
    int32_t n_iter;
} nbsi_fit;

/* Synthesized beam of every channel of a plan: the image of unit Stokes-I visibilities on the
 * plan's baselines (its point-spread function, same imager and uv cuts) fitted as above with
 * half = NBSI_BEAM_HALF at the image centre.  beam: device double [n_chan][3] (FWHM major,
 * minor in pixels, pa; NaN if the fit fails), 8-byte aligned.  Asynchronous on the context's
 * stream; uses context scratch for one imager chunk of the point-spread function. */
int nbsi_beam(nbsi_ctx *ctx, const nbsi_image_plan *plan, double *beam);

/* Stage II over candidates on an image cube img [n_chan][n_pix][n_pix] float32 (device,
 * 16-byte aligned; shape limits of nbsi_detect): cands [n_cand] device nbsi_cand (x, y, c used),
 * beam device double [n_chan][3] (e.g. from nbsi_beam), 2 <= half <= NBSI_S2_MAX_HALF,
 * ext_factor > 0, noise_k >= 1, 0 <= n_cand <= NBSI_S2_MAX_CANDS; out [n_cand] device nbsi_fit
 * (fields NaN where no fit was made).  Asynchronous on the context's stream. */
int nbsi_stage2(nbsi_ctx *ctx, const float *img, int n_chan, int n_pix, const nbsi_cand *cands, int n_cand,
                const double *beam, int half, double ext_factor, double noise_k, nbsi_fit *out);

/*
 * Batched sub-bands (Sec. 2.1: the band is processed as independent batches of fine channels;
 * Sec. 2.6: re-processing with other FFT lengths and integrations).  Each sub-band is one coarse
 * channel's voltages with its own FFT length, integration count, kept channels and image size;
 * nbsi_batch_run channelizes, correlates and images all of them (each stage one launch
 * over a task table spanning the sub-bands, grouped only where kernel shapes differ), with the
 * same results as the per-sub-band calls above (bit-identical spectra, visibilities and images).
 */
typedef struct {
    const int8_t *volt;          /* [n_in][n_spec * n_fft][2] int8, n_in = 2 n_ant */
    const float *gain;           /* [n_in] requantisation gains */
    int n_fft, n_spec, chan0, n_chan;
    const double *freq_hz_host;  /* [n_chan] sky frequency of each kept channel (host) */
    int n_pix;                   /* image size (NBSI_IMAGE_GRID) */
    int8_t *spec_q;              /* out [n_chan][n_in][2][n_spec] */
    int32_t *vis;                /* out [n_chan][n_in (n_in+1)/2][2] */
    float *img;                  /* out [n_chan][n_pix][n_pix] */
} nbsi_subband;

typedef struct nbsi_batch nbsi_batch;

#define NBSI_BATCH_GRAPH 1     /* capture the launches into a hipGraph on the first run, replay after */
#define NBSI_BATCH_AUTOTUNE 2  /* time correlator variants and gridding tiles per shape at plan time */
#define NBSI_BATCH_GRID_TALL 4 /* grid with the 32-cell-per-thread tile everywhere (no gridding tuning) */
#define NBSI_BATCH_OVERLAP 8   /* pipeline the sub-bands: while sub-band s is correlated and imaged on
                                  an auxiliary stream of the batch, sub-band s + 1 is channelized
                                  (stages launched per sub-band, directly: NBSI_BATCH_GRAPH is not
                                  used with it; same outputs, bit for bit) */

/*
 * Plan a batch: validates every sub-band, builds its imaging plan, allocates the batch's
 * scratch (staging, Stokes-I gathers, row-transform intermediates; kept until destroy) and the
 * task tables.  With NBSI_BATCH_AUTOTUNE the plan runs the stages once to time the candidates
 * (this writes the sub-bands' outputs); choices are read from and added to the text file
 * tune_cache_path (may be NULL).  The batch runs on its own stream, ordered after and before the
 * context's stream with events.  Not thread-safe; one batch at a time per context.
 */
int nbsi_batch_plan(nbsi_ctx *ctx, const double *ant_xyz_host, int n_ant, const nbsi_subband *sb, int n_sb,
                    int precision, int flags, const char *tune_cache_path, nbsi_batch **plan);
int nbsi_batch_run(nbsi_batch *plan);
/* JSON text of the per-sub-band choices (correlator variant, gridding tile) into buf[len]. */
int nbsi_batch_describe(const nbsi_batch *plan, char *buf, int len);
int nbsi_batch_destroy(nbsi_batch *plan);


/*
 * Learned candidate classifier (stands in for the paper's Stage II screen of Stage I
 * candidates, Sec. 2.4, which rejects extended, horizon-hugging and image-wide structures; the
 * network itself is not in the paper).  A candidate is scored from a stamp of the detector's SNR
 * cube: 33 channels (c - 16 .. c + 16) by 9 x 9 pixels centred on (c, y, x), zero outside the
 * cube, FP16, layout [33][9][9].  Network: conv3x3(33->32)-ReLU-conv3x3(32->64)-ReLU-
 * conv3x3(64->32)-ReLU, zero padding 1, global average pool, linear(32->1) -> logit (label 1 =
 * sky-localised narrowband tone).  Loss: mean binary cross-entropy on the logit.  Products run
 * on FP16 matrix cores with FP32 accumulation; master weights, Adam moments and gradients are
 * FP32.  Parameters are one float vector of NBSI_NET_NPARAM entries in the order
 *   W1[32][33][3][3], b1[32], W2[64][32][3][3], b2[64], W3[32][64][3][3], b3[32], w4[32], b4[1]
 * (a convolution is a cross-correlation: Z[o][y][x] = b[o] + sum W[o][i][dy][dx] X[i][y+dy-1][x+dx-1]).
 * All calls are asynchronous on the context's stream unless stated otherwise.
 */
#define NBSI_STAMP_CHANNELS 33
#define NBSI_STAMP_PIXELS 9
#define NBSI_NET_NPARAM 46529
#define NBSI_NET_MAX_BATCH 8192

typedef struct nbsi_net nbsi_net;

/* Stamps of cube [n_chan][n_pix][n_pix] float32 (device) around cands[n] (device, nbsi_cand)
 * into stamps [n][33][9][9] (device, FP16 bits, round to nearest even, saturating at +-65504). */
int nbsi_stamps(nbsi_ctx *ctx, const float *cube, int n_chan, int n_pix, const nbsi_cand *cands, int n,
                uint16_t *stamps);
/* Network with the given parameters (host, NBSI_NET_NPARAM floats) and device buffers for
 * batches of up to max_batch stamps (<= NBSI_NET_MAX_BATCH).  Adam state starts at zero. */
int nbsi_net_create(nbsi_ctx *ctx, const float *params_host, int max_batch, nbsi_net **net);
int nbsi_net_destroy(nbsi_net *net);
/* Replace the parameters (host) and reset Adam's moments and step count; blocking. */
int nbsi_net_set_params(nbsi_net *net, const float *params_host);
/* Copy the FP32 master parameters to the host; blocking. */
int nbsi_net_get_params(nbsi_net *net, float *params_host);
/* Logits of a batch: stamps [n_stamps][33][9][9] FP16 (device, 8-byte aligned); the batch is
 * stamps index[0..n) (device int32; out-of-range entries read as empty stamps) or, with
 * index NULL, the first n stamps (n <= n_stamps).  logits: device float [n]. */
int nbsi_net_forward(nbsi_net *net, const uint16_t *stamps, int n_stamps, const int32_t *index, int n, float *logits);
/* Mean loss and gradient of a batch: labels (device float, 0 or 1) are indexed like the stamps;
 * loss: device float [1] or NULL; grad: device float [NBSI_NET_NPARAM] or NULL (the network's
 * own gradient buffer, used by nbsi_net_adam with grad NULL). */
int nbsi_net_grad(nbsi_net *net, const uint16_t *stamps, int n_stamps, const int32_t *index, const float *labels, int n,
                  float *loss, float *grad);
/* One Adam step (Kingma & Ba) on the master parameters with the device gradient grad (NULL: the
 * network's own buffer); the step count advances by one. */
int nbsi_net_adam(nbsi_net *net, const float *grad, float lr, float beta1, float beta2, float eps);
/* nbsi_net_grad into the network's buffer, then nbsi_net_adam(lr, 0.9, 0.999, 1e-8). */
int nbsi_net_train_step(nbsi_net *net, const uint16_t *stamps, int n_stamps, const int32_t *index, const float *labels,
                        int n, float lr, float *loss);

#ifdef __cplusplus
}
#endif

#endif /* NBSI_H */
