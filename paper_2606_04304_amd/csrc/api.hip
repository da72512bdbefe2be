// Host side of the C ABI: validation, context and scratch management, imaging plans.
#include "internal.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

int channelize_log_m(int log_n, int n_chan);
int detect_ppw(int n_chan);

// Fixed workspace of the no-allocation detector entry point: one copy per GPU, held until the
// process ends.  Host code never passes `scratch` itself (on the host it names a stand-in, not
// device memory); it uses the address hipGetSymbolAddress returns on each device, resolved
// once per device by nbsi_create with that device current.  Layout: candidate counter, the
// per-channel statistics of up to 32,768 channels, NBSI_DETECT_NOALLOC_MAX_CANDS candidates
// and as many sort keys.
constexpr size_t NOALLOC_OFF_COUNTER = 0;
constexpr size_t NOALLOC_OFF_STATS = 256;
constexpr size_t NOALLOC_OFF_CAND = NOALLOC_OFF_STATS + sizeof(float2) * 32768;
constexpr size_t NOALLOC_OFF_KEYS = NOALLOC_OFF_CAND + sizeof(nbsi_cand) * (size_t)NBSI_DETECT_NOALLOC_MAX_CANDS;
constexpr size_t NOALLOC_END = NOALLOC_OFF_KEYS + sizeof(unsigned long long) * (size_t)NBSI_DETECT_NOALLOC_MAX_CANDS;
static_assert(NOALLOC_END == NBSI_DETECT_NOALLOC_BYTES, "workspace layout");
static_assert(NOALLOC_OFF_CAND % 256 == 0 && NOALLOC_OFF_KEYS % 256 == 0, "workspace alignment");

static __device__ __align__(256) unsigned char scratch[NBSI_DETECT_NOALLOC_BYTES];

constexpr int NBSI_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[NBSI_MAX_DEVICES] = {};

// Resolve this device's copy of the workspace (the device must be current).
static int resolve_noalloc_scratch(int device) {
    if (device < 0 || device >= NBSI_MAX_DEVICES) return NBSI_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return NBSI_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return NBSI_EHIP;
    g_scratch_ptr[device] = ptr;
    return NBSI_OK;
}

namespace {

constexpr double C_LIGHT = 299792458.0;

bool is_pow2(long n) { return n > 0 && (n & (n - 1)) == 0; }
int ilog2(long n) {
    int l = 0;
    while ((1L << l) < n) l++;
    return l;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n).
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; i++) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = 0.0;
            for (int k = 1; k <= n; k++) {
                const double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
            }
            dp = n * (z * p0 - p1) / (z * z - 1.0);
            const double dz = p0 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

}  // namespace

int nbsi_fail(nbsi_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->last_error = msg;
    return code;
}

int nbsi_scratch(nbsi_ctx *ctx, int slot, size_t bytes, void **ptr) {
    if (bytes == 0) bytes = 256;
    if (ctx->scratch_size[slot] < bytes) {
        if (ctx->scratch[slot]) {
            // the old buffer may still be read by queued work of this stream
            if (hipStreamSynchronize(ctx->stream) != hipSuccess) return nbsi_fail(ctx, NBSI_EHIP, "stream sync failed");
            (void)hipFree(ctx->scratch[slot]);
            ctx->scratch[slot] = nullptr;
            ctx->scratch_size[slot] = 0;
        }
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess || !p)
            return nbsi_fail(ctx, NBSI_ENOMEM, "scratch allocation of " + std::to_string(bytes) + " bytes failed");
        ctx->scratch[slot] = p;
        ctx->scratch_size[slot] = bytes;
    }
    *ptr = ctx->scratch[slot];
    return NBSI_OK;
}

namespace {

// the auxiliary stream (non-blocking, default priority) and the stage events of a context
int nbsi_aux_stream(nbsi_ctx *ctx) {
    if (ctx->aux) return NBSI_OK;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
        return nbsi_fail(ctx, NBSI_EHIP, "auxiliary stream creation failed");
    for (int k = 0; k <= NBSI_MAX_STAGES; k++)
        if (hipEventCreateWithFlags(&ctx->ev_stage[k], hipEventDisableTiming) != hipSuccess) {
            for (int j = 0; j < k; j++) (void)hipEventDestroy(ctx->ev_stage[j]);
            for (int j = 0; j <= NBSI_MAX_STAGES; j++) ctx->ev_stage[j] = nullptr;
            (void)hipStreamDestroy(s);
            return nbsi_fail(ctx, NBSI_EHIP, "stage event creation failed");
        }
    ctx->aux = s;
    return NBSI_OK;
}

int check_image_stokes(nbsi_ctx *ctx, const nbsi_image_plan *plan, int precision, const char *who) {
    if (plan->device != ctx->device) return nbsi_fail(ctx, NBSI_EINVAL, std::string(who) + ": plan built on another device");
    if (plan->method != NBSI_IMAGE_GRID) return nbsi_fail(ctx, NBSI_EINVAL, std::string(who) + ": plan must be a gridding plan");
    if (precision != NBSI_PREC_FP32 && precision != NBSI_PREC_FP16 && precision != NBSI_PREC_BF16)
        return nbsi_fail(ctx, NBSI_EINVAL, std::string(who) + ": bad precision");
    return NBSI_OK;
}

// The imager runs over channel chunks whose row-pass intermediate stays in the last-level cache.
size_t image_stokes_per_chan(const nbsi_image_plan *plan) { return (size_t)plan->n_pix * plan->n_pix * sizeof(float2); }

int image_stokes_chunk(const nbsi_image_plan *plan) {
    return (int)std::max<size_t>(1, std::min<size_t>(plan->n_chan, IMAGE_CHUNK_BYTES / image_stokes_per_chan(plan)));
}

// Images of channels [c_begin, c_end) (c_begin a multiple of the chunk) from their Stokes-I rows.
hipError_t image_stokes_range(const nbsi_image_plan *plan, const float *stokes_i, int precision, float2 *inter,
                              float *img, int c_begin, int c_end, hipStream_t st, unsigned *flags) {
    const int chunk = image_stokes_chunk(plan);
    const float2 *sv = reinterpret_cast<const float2 *>(stokes_i);
    for (int c0 = c_begin; c0 < c_end; c0 += chunk) {
        nbsi_image_plan sub = *plan;
        sub.n_chan = std::min(chunk, c_end - c0);
        sub.d_freq = plan->d_freq + c0;
        sub.d_nb = plan->d_nb + c0;
        if (plan->d_inb) sub.d_inb = plan->d_inb + (size_t)c0 * ((plan->n_pairs + 31) >> 5);
        const hipError_t e = launch_image_grid_stokes(&sub, sv + (size_t)c0 * plan->n_pairs, precision, inter,
                                                      img + (size_t)c0 * plan->n_pix * plan->n_pix, st, flags);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Workspace of the detector when the caller's call may not allocate: stats, the candidate
// buffer (cap entries), sort keys for cap entries and the candidate counter.
struct DetectWs {
    float *stats = nullptr;
    nbsi_cand *cand = nullptr;
    unsigned long long *keys = nullptr;
    int *counter = nullptr;
    int cap = 0;
};

// nbsi_detect with context scratch (ws null; grown when the candidates overflow it) or with a
// fixed workspace (ws set; more candidates than it holds is an error, nothing is allocated).
int detect_run(nbsi_ctx *ctx, const float *img, int n_chan, int n_pix, int mode, float thresh, float *snr,
               nbsi_cand *out, int max_out, int *n_out, const DetectWs *ws, const char *who) {
    if (!ctx) return NBSI_EINVAL;
    const std::string w(who);
    int rc = nbsi_check_detect(n_chan, n_pix, mode, max_out);
    if (rc) return nbsi_fail(ctx, rc, w + ": bad shape");
    if (!img || !n_out || (max_out > 0 && !out)) return nbsi_fail(ctx, NBSI_EINVAL, w + ": null pointer");
    if (!aligned16(img) || (snr && !aligned16(snr)) || (out && !aligned16(out)))
        return nbsi_fail(ctx, NBSI_EINVAL, w + ": misaligned pointer");
    DeviceGuard g(ctx->device);
    void *stats = ws ? (void *)ws->stats : nullptr;
    if (!ws && (rc = nbsi_scratch(ctx, SLOT_DET_STATS, sizeof(float2) * n_chan, &stats))) return rc;
    int *counter = ws ? ws->counter : ctx->d_counter;
    NBSI_TRY_HIP(ctx, launch_detect_stats(img, n_chan, n_pix, mode, (float *)stats, ctx->stream));
    int cap = ws ? ws->cap : (int)std::max<size_t>(65536, ctx->scratch_size[SLOT_DET_CAND] / sizeof(nbsi_cand));
    int count = 0;
    void *cand = nullptr;
    for (int attempt = 0; attempt < 2; attempt++) {
        cand = ws ? (void *)ws->cand : nullptr;
        if (!ws && (rc = nbsi_scratch(ctx, SLOT_DET_CAND, sizeof(nbsi_cand) * (size_t)cap, &cand))) return rc;
        NBSI_TRY_HIP(ctx, hipMemsetAsync(counter, 0, sizeof(int), ctx->stream));
        NBSI_TRY_HIP(ctx, launch_detect_scan(img, n_chan, n_pix, mode, (const float *)stats, thresh, snr,
                                             (nbsi_cand *)cand, cap, counter, ctx->stream, ctx->d_flags));
        // the usual few candidates are sorted before the count comes back: one wait per call
        NBSI_TRY_HIP(ctx, launch_detect_sort_small_dev((const nbsi_cand *)cand, counter, cap, n_chan, n_pix, out,
                                                       max_out, ctx->stream));
        NBSI_TRY_HIP(ctx, hipMemcpyAsync(&count, counter, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        NBSI_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (count <= cap) break;
        if (ws)
            return nbsi_fail(ctx, NBSI_EOVERFLOW,
                             w + ": " + std::to_string(count) + " candidates, more than the fixed workspace's " +
                                 std::to_string(cap) + " (use nbsi_detect)");
        if (count > (1 << 24)) return nbsi_fail(ctx, NBSI_EOVERFLOW, w + ": more than 2^24 candidates");
        cap = count;
    }
    *n_out = count;
    const int n_write = std::min(count, max_out);
    if (count > detect_sort_small_max() && n_write > 0) {
        int n_pow2 = 1;
        while (n_pow2 < count) n_pow2 <<= 1;
        void *keys = ws ? (void *)ws->keys : nullptr;
        if (!ws && (rc = nbsi_scratch(ctx, SLOT_DET_KEYS, sizeof(unsigned long long) * n_pow2, &keys))) return rc;
        NBSI_TRY_HIP(ctx, launch_detect_sort((nbsi_cand *)cand, count, (unsigned long long *)keys, n_chan, n_pix, out,
                                             n_write, ctx->stream));
        NBSI_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    return count > max_out ? NBSI_ETRUNC : NBSI_OK;
}

}  // namespace

extern "C" {

int nbsi_version(void) { return 1; }

const char *nbsi_strerror(int status) {
    switch (status) {
        case NBSI_OK: return "ok";
        case NBSI_EINVAL: return "invalid argument";
        case NBSI_EOVERFLOW: return "result would overflow its type";
        case NBSI_ENOMEM: return "out of device memory";
        case NBSI_EHIP: return "HIP runtime error";
        case NBSI_ETRUNC: return "output truncated";
        case NBSI_EUNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

int nbsi_check_channelize(int n_in, int n_fft, int n_spec, int chan0, int n_chan) {
    if (n_in < 1 || n_chan < 1) return NBSI_EINVAL;
    if (!is_pow2(n_fft) || n_fft < 256 || n_fft > (1 << 18)) return NBSI_EINVAL;
    if (n_spec < 1) return NBSI_EINVAL;
    if (n_spec > NBSI_MAX_SPEC) return NBSI_EOVERFLOW;
    if (chan0 < 0 || chan0 + (long)n_chan > n_fft || n_chan > 16384) return NBSI_EINVAL;
    if ((long)n_in * n_spec > 0x7fffffffL) return NBSI_EINVAL;
    return NBSI_OK;
}

int nbsi_check_correlate(int n_chan, int n_in, int n_spec) {
    if (n_chan < 1 || n_in < 1 || n_spec < 1) return NBSI_EINVAL;
    if (n_spec > NBSI_MAX_SPEC) return NBSI_EOVERFLOW;
    if (n_in > 8192) return NBSI_EINVAL;
    return NBSI_OK;
}

int nbsi_check_image(int n_chan, int n_ant, int n_pix, int method, int precision, double uv_min,
                     double uv_max) {
    if (n_chan < 1 || n_ant < 2 || n_ant > 4096) return NBSI_EINVAL;
    if (n_pix < 8 || n_pix > 1024 || (n_pix & 7)) return NBSI_EINVAL;
    if (method != NBSI_IMAGE_DFT && method != NBSI_IMAGE_GRID) return NBSI_EINVAL;
    if (method == NBSI_IMAGE_GRID && (!is_pow2(n_pix) || n_pix < 64)) return NBSI_EINVAL;
    if (precision != NBSI_PREC_FP32 && precision != NBSI_PREC_FP16 && precision != NBSI_PREC_BF16)
        return NBSI_EINVAL;
    if (!(uv_min >= 0.0) || !(uv_max >= uv_min)) return NBSI_EINVAL;
    return NBSI_OK;
}

int nbsi_check_detect(int n_chan, int n_pix, int mode, int max_out) {
    if (n_chan < 3 || n_chan > 32768) return NBSI_EINVAL;
    if (n_pix < 8 || n_pix > 1024 || (n_pix & 7)) return NBSI_EINVAL;
    if (mode != NBSI_DETECT_PER_PIXEL && mode != NBSI_DETECT_PER_IMAGE) return NBSI_EINVAL;
    if (max_out < 0) return NBSI_EINVAL;
    return NBSI_OK;
}

const char *nbsi_correlate_kernel(int n_in, int n_spec) {
    switch (correlate_default_variant(n_in, n_spec)) {
        case CORR_VARIANT_CHAN32: return "correlate_i8_chan_kernel<32>";
        case CORR_VARIANT_CHAN64: return "correlate_i8_chan_kernel<64>";
        default:  // 16-byte row strides (other integrations are repacked to one first)
            return n_spec >= PIPE_BIG_T ? "correlate_i8_pipe_kernel<256>" : "correlate_i8_pipe_kernel<128>";
    }
}

int nbsi_create(nbsi_ctx **out, int device, void *stream) {
    if (!out) return NBSI_EINVAL;
    *out = nullptr;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || device < 0 || device >= n_dev) return NBSI_EHIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return NBSI_EHIP;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return NBSI_EUNSUPPORTED;
    nbsi_ctx *ctx = new (std::nothrow) nbsi_ctx();
    if (!ctx) return NBSI_ENOMEM;
    ctx->device = device;
    ctx->stream = (hipStream_t)stream;
    DeviceGuard g(device);
    if (!g.ok || hipMalloc(&ctx->d_counter, 256) != hipSuccess) {
        delete ctx;
        return NBSI_EHIP;
    }
    if (hipMalloc(&ctx->d_flags, 256) != hipSuccess || hipMemset(ctx->d_flags, 0, 256) != hipSuccess) {
        if (ctx->d_flags) (void)hipFree(ctx->d_flags);
        (void)hipFree(ctx->d_counter);
        delete ctx;
        return NBSI_EHIP;
    }
    if (const int rs = resolve_noalloc_scratch(device)) {
        (void)hipFree(ctx->d_flags);
        (void)hipFree(ctx->d_counter);
        delete ctx;
        return rs;
    }
    *out = ctx;
    return NBSI_OK;
}

int nbsi_destroy(nbsi_ctx *ctx) {
    if (!ctx) return NBSI_EINVAL;
    DeviceGuard g(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->aux) {
        (void)hipStreamSynchronize(ctx->aux);
        for (int k = 0; k <= NBSI_MAX_STAGES; k++) (void)hipEventDestroy(ctx->ev_stage[k]);
        (void)hipStreamDestroy(ctx->aux);
    }
    if (ctx->ev_switch) (void)hipEventDestroy(ctx->ev_switch);
    for (int s = 0; s < 16; s++)
        if (ctx->scratch[s]) (void)hipFree(ctx->scratch[s]);
    if (ctx->d_counter) (void)hipFree(ctx->d_counter);
    if (ctx->d_flags) (void)hipFree(ctx->d_flags);
    delete ctx;
    return NBSI_OK;
}

int nbsi_set_stream(nbsi_ctx *ctx, void *stream) {
    if (!ctx) return NBSI_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (s == ctx->stream) return NBSI_OK;
    // the context's scratch is shared by all its calls: work enqueued on the new stream waits
    // for everything the context enqueued before (its old stream and auxiliary stream)
    DeviceGuard g(ctx->device);
    if (!ctx->ev_switch) NBSI_TRY_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_switch, hipEventDisableTiming));
    NBSI_TRY_HIP(ctx, hipEventRecord(ctx->ev_switch, ctx->stream));
    NBSI_TRY_HIP(ctx, hipStreamWaitEvent(s, ctx->ev_switch, 0));
    if (ctx->aux) {
        NBSI_TRY_HIP(ctx, hipEventRecord(ctx->ev_switch, ctx->aux));
        NBSI_TRY_HIP(ctx, hipStreamWaitEvent(s, ctx->ev_switch, 0));
    }
    ctx->stream = s;
    return NBSI_OK;
}

const char *nbsi_last_error(const nbsi_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

int nbsi_synchronize(nbsi_ctx *ctx) {
    if (!ctx) return NBSI_EINVAL;
    DeviceGuard g(ctx->device);
    NBSI_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return NBSI_OK;
}

int nbsi_status(nbsi_ctx *ctx, uint32_t *flags_host) {
    if (!ctx || !flags_host) return NBSI_EINVAL;
    DeviceGuard g(ctx->device);
    NBSI_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->aux) NBSI_TRY_HIP(ctx, hipStreamSynchronize(ctx->aux));
    unsigned f = 0;
    NBSI_TRY_HIP(ctx, hipMemcpyAsync(&f, ctx->d_flags, sizeof(f), hipMemcpyDeviceToHost, ctx->stream));
    NBSI_TRY_HIP(ctx, hipMemsetAsync(ctx->d_flags, 0, sizeof(f), ctx->stream));
    NBSI_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *flags_host = f;
    return NBSI_OK;
}

int nbsi_channelize(nbsi_ctx *ctx, const int8_t *volt, int n_in, int n_fft, int n_spec, int chan0,
                    int n_chan, const float *gain, int8_t *spec_q, float *spec_f) {
    if (!ctx) return NBSI_EINVAL;
    int rc = nbsi_check_channelize(n_in, n_fft, n_spec, chan0, n_chan);
    if (rc) return nbsi_fail(ctx, rc, "nbsi_channelize: bad shape");
    if (!volt || !gain || (!spec_q && !spec_f)) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_channelize: null pointer");
    if (!aligned16(volt) || !aligned16(gain) || (spec_q && !aligned16(spec_q)) || (spec_f && !aligned16(spec_f)))
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_channelize: pointers must be 16-byte aligned");
    DeviceGuard g(ctx->device);
    const int log_n = ilog2(n_fft);
    const int klo = (chan0 + n_fft / 2) & (n_fft - 1);
    const size_t cells = (size_t)n_in * n_spec * n_chan;
    void *sq = nullptr, *sf = nullptr;
    if (spec_q && (rc = nbsi_scratch(ctx, SLOT_CHAN_STAGE_Q, cells * 2, &sq))) return rc;
    if (spec_f && (rc = nbsi_scratch(ctx, SLOT_CHAN_STAGE_F, cells * 8, &sf))) return rc;
    NBSI_TRY_HIP(ctx, launch_channelize(volt, n_in, log_n, n_spec, klo, n_chan, gain, (int8_t *)sq, (float *)sf,
                                        ctx->stream, ctx->d_flags));
    if (spec_q) NBSI_TRY_HIP(ctx, launch_corner_turn_q((int8_t *)sq, n_in, n_spec, n_chan, spec_q, ctx->stream));
    if (spec_f) NBSI_TRY_HIP(ctx, launch_corner_turn_f((float *)sf, n_in, n_spec, n_chan, spec_f, ctx->stream));
    return NBSI_OK;
}

int nbsi_correlate(nbsi_ctx *ctx, const int8_t *spec_q, int n_chan, int n_in, int n_spec, int32_t *vis) {
    if (!ctx) return NBSI_EINVAL;
    int rc = nbsi_check_correlate(n_chan, n_in, n_spec);
    if (rc) return nbsi_fail(ctx, rc, "nbsi_correlate: bad shape");
    if (!spec_q || !vis) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_correlate: null pointer");
    if (!aligned16(spec_q) || !aligned16(vis)) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_correlate: misaligned pointer");
    DeviceGuard g(ctx->device);
    void *pad = nullptr;
    if (const size_t pb = correlate_pad_bytes(n_chan, n_in, n_spec))
        if ((rc = nbsi_scratch(ctx, SLOT_CORR_PAD, pb, &pad))) return rc;
    NBSI_TRY_HIP(ctx, launch_correlate_i8(spec_q, n_chan, n_in, n_spec, vis, ctx->stream, StokesOut(), (int8_t *)pad));
    return NBSI_OK;
}

int nbsi_correlate_stokes(nbsi_ctx *ctx, const int8_t *spec_q, int n_chan, int n_in, int n_spec,
                          const nbsi_image_plan *plan, int32_t *vis, float *stokes_i) {
    if (!ctx) return NBSI_EINVAL;
    int rc = nbsi_check_correlate(n_chan, n_in, n_spec);
    if (rc) return nbsi_fail(ctx, rc, "nbsi_correlate_stokes: bad shape");
    if (!spec_q || !vis || !plan || !stokes_i) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_correlate_stokes: null pointer");
    if (!aligned16(spec_q) || !aligned16(vis) || !aligned16(stokes_i))
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_correlate_stokes: misaligned pointer");
    if (plan->device != ctx->device) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_correlate_stokes: plan built on another device");
    if (plan->method != NBSI_IMAGE_GRID || n_in != 2 * plan->n_ant || n_chan != plan->n_chan)
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_correlate_stokes: plan must be a gridding plan of n_in / 2 antennas and n_chan channels");
    DeviceGuard g(ctx->device);
    StokesOut so;
    so.mask = plan->d_tmask;
    so.base = plan->d_tbase;
    so.out = reinterpret_cast<float2 *>(stokes_i);
    so.n_pairs = plan->n_pairs;
    void *pad = nullptr;
    if (const size_t pb = correlate_pad_bytes(n_chan, n_in, n_spec))
        if ((rc = nbsi_scratch(ctx, SLOT_CORR_PAD, pb, &pad))) return rc;
    NBSI_TRY_HIP(ctx, launch_correlate_i8(spec_q, n_chan, n_in, n_spec, vis, ctx->stream, so, (int8_t *)pad));
    return NBSI_OK;
}

int nbsi_correlate_cal(nbsi_ctx *ctx, const int8_t *spec_q, int n_chan, int n_in, int n_spec, const float *cal,
                       float *vis_cal) {
    if (!ctx) return NBSI_EINVAL;
    int rc = nbsi_check_correlate(n_chan, n_in, n_spec);
    if (rc) return nbsi_fail(ctx, rc, "nbsi_correlate_cal: bad shape");
    if (!spec_q || !cal || !vis_cal) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_correlate_cal: null pointer");
    if (!aligned16(spec_q) || !aligned16(vis_cal) || ((uintptr_t)cal & 7u))
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_correlate_cal: misaligned pointer");
    DeviceGuard g(ctx->device);
    void *pad = nullptr;
    if (const size_t pb = correlate_pad_bytes(n_chan, n_in, n_spec))
        if ((rc = nbsi_scratch(ctx, SLOT_CORR_PAD, pb, &pad))) return rc;
    NBSI_TRY_HIP(ctx, launch_correlate_i8(spec_q, n_chan, n_in, n_spec, reinterpret_cast<int32_t *>(vis_cal),
                                          ctx->stream, StokesOut(), (int8_t *)pad,
                                          reinterpret_cast<const float2 *>(cal)));
    return NBSI_OK;
}

int nbsi_correlate_f32(nbsi_ctx *ctx, const float *spec_f, int n_chan, int n_in, int n_spec, float *vis) {
    if (!ctx) return NBSI_EINVAL;
    int rc = nbsi_check_correlate(n_chan, n_in, n_spec);
    if (rc == NBSI_EOVERFLOW) rc = NBSI_OK;  // float accumulation has no int32 bound
    if (rc) return nbsi_fail(ctx, rc, "nbsi_correlate_f32: bad shape");
    if (!spec_f || !vis) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_correlate_f32: null pointer");
    if (!aligned16(spec_f) || !aligned16(vis))
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_correlate_f32: misaligned pointer");
    DeviceGuard g(ctx->device);
    NBSI_TRY_HIP(ctx, launch_correlate_f32(spec_f, n_chan, n_in, n_spec, vis, ctx->stream));
    return NBSI_OK;
}

}  // extern "C"

// Build an imaging plan; ge selects the gridding tile (256 ge grid cells per workgroup).
int image_plan_build(nbsi_ctx *ctx, const double *ant_xyz_host, int n_ant, const double *freq_hz_host, int n_chan,
                     int n_pix, int method, double uv_min, double uv_max, int ge, nbsi_image_plan **out) {
    if (!ctx || !out) return NBSI_EINVAL;
    *out = nullptr;
    int rc = nbsi_check_image(n_chan, n_ant, n_pix, method, NBSI_PREC_FP32, uv_min, uv_max);
    if (rc) return nbsi_fail(ctx, rc, "nbsi_image_plan_create: bad shape or parameters");
    if (!ant_xyz_host || !freq_hz_host) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_image_plan_create: null pointer");
    double nu_min = freq_hz_host[0], nu_max = freq_hz_host[0];
    for (int c = 0; c < n_chan; c++) {
        if (!(freq_hz_host[c] > 0.0) || !isfinite(freq_hz_host[c]))
            return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_image_plan_create: frequencies must be positive");
        nu_min = std::min(nu_min, freq_hz_host[c]);
        nu_max = std::max(nu_max, freq_hz_host[c]);
    }
    DeviceGuard g(ctx->device);
    nbsi_image_plan *p = new (std::nothrow) nbsi_image_plan();
    if (!p) return NBSI_ENOMEM;
    p->device = ctx->device;
    p->n_ant = n_ant;
    p->n_chan = n_chan;
    p->n_pix = n_pix;
    p->method = method;
    p->ge = ge;
    p->uv_min = uv_min;
    p->uv_max = uv_max;

    // Candidate pairs: every pair that can be in B for some channel frequency (1e-9 slack; the
    // kernels apply the exact per-channel test).
    const double slack = 1e-9;
    const double U = (double)(n_pix - 5) * 0.25;
    const int M = 2 * n_pix;
    std::vector<int2> pairs;
    std::vector<double2> dxy;
    std::vector<int> lo_row, hi_row;
    for (int a = 0; a < n_ant; a++)
        for (int b = 0; b < a; b++) {
            const double dx = ant_xyz_host[3 * a] - ant_xyz_host[3 * b];
            const double dy = ant_xyz_host[3 * a + 1] - ant_xyz_host[3 * b + 1];
            const double r = sqrt(dx * dx + dy * dy);
            if (r * nu_max / C_LIGHT < uv_min * (1 - slack) - 1e-12) continue;
            if (r * nu_min / C_LIGHT > uv_max * (1 + slack) + 1e-12) continue;
            if (method == NBSI_IMAGE_GRID) {
                if (fabs(dx) * nu_min / C_LIGHT > U * (1 + slack)) continue;
                if (fabs(dy) * nu_min / C_LIGHT > U * (1 + slack)) continue;
                const double v1 = dy * nu_min / C_LIGHT * 4.0 + M / 2, v2 = dy * nu_max / C_LIGHT * 4.0 + M / 2;
                lo_row.push_back(std::max(0, (int)floor(std::min(v1, v2)) - 4));
                hi_row.push_back(std::min(M - 1, (int)floor(std::max(v1, v2)) + 5));
            }
            pairs.push_back(make_int2(a, b));
            dxy.push_back(make_double2(dx, dy));
        }
    // Order the candidates by 8 x 8 antenna block (packed lower-triangle block order), then by
    // position within the block: the correlator's epilogue finds a pair's index from its block's
    // bit mask and base (one 32 x 32 tile of the correlation matrix is one such block).
    const int n_blk = (n_ant + 7) / 8;
    const size_t n_tiles = (size_t)n_blk * (n_blk + 1) / 2;
    auto tile_of = [](int a, int b) { return (size_t)(a / 8) * (a / 8 + 1) / 2 + (size_t)(b / 8); };
    auto bit_of = [](int a, int b) { return (a % 8) * 8 + b % 8; };
    {
        std::vector<int> ord(pairs.size());
        for (size_t k = 0; k < ord.size(); k++) ord[k] = (int)k;
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
            const size_t tx = tile_of(pairs[x].x, pairs[x].y), ty = tile_of(pairs[y].x, pairs[y].y);
            return tx != ty ? tx < ty : bit_of(pairs[x].x, pairs[x].y) < bit_of(pairs[y].x, pairs[y].y);
        });
        std::vector<int2> p2(pairs.size());
        std::vector<double2> d2(dxy.size());
        std::vector<int> l2(lo_row.size()), h2(hi_row.size());
        for (size_t k = 0; k < ord.size(); k++) {
            p2[k] = pairs[ord[k]];
            d2[k] = dxy[ord[k]];
            if (!lo_row.empty()) {
                l2[k] = lo_row[ord[k]];
                h2[k] = hi_row[ord[k]];
            }
        }
        pairs.swap(p2);
        dxy.swap(d2);
        lo_row.swap(l2);
        hi_row.swap(h2);
    }
    std::vector<unsigned long long> tmask(n_tiles, 0ull);
    std::vector<int> tbase(n_tiles, 0);
    for (const int2 &pr : pairs) tmask[tile_of(pr.x, pr.y)] |= 1ull << bit_of(pr.x, pr.y);
    for (size_t t = 0, run = 0; t < n_tiles; t++) {
        tbase[t] = (int)run;
        run += (size_t)__builtin_popcountll(tmask[t]);
    }
    p->n_pairs = (int)pairs.size();

    std::vector<int> band_off, band_items;
    std::vector<float> corr;
    if (method == NBSI_IMAGE_GRID) {
        // The image is the real part of the grid's transform, i.e. half the transform of the
        // Hermitian grid h(u, v) = g(u, v) + conj g(-u, -v): every pair is gridded at +(u, v)
        // with V and at -(u, v) with conj V, and only the rows v >= 0 (array rows M/2 .. M-1)
        // are gridded and row-transformed; the column pass recovers v < 0 by symmetry.  Items
        // are 2 k + mirrored.
        p->band_rows = 256 * ge / M;
        p->n_bands = (M / 2) / p->band_rows;
        std::vector<std::vector<int>> bins(p->n_bands);
        for (int k = 0; k < p->n_pairs; k++)
            for (int mir = 0; mir < 2; mir++) {
                const int lo = mir ? M - hi_row[k] : lo_row[k], hi = mir ? M - lo_row[k] : hi_row[k];
                if (hi < M / 2) continue;
                const int b0 = (std::max(lo, M / 2) - M / 2) / p->band_rows;
                const int b1 = (std::min(hi, M - 1) - M / 2) / p->band_rows;
                for (int bnd = b0; bnd <= b1; bnd++) bins[bnd].push_back(2 * k + mir);
            }
        band_off.push_back(0);
        for (int bnd = 0; bnd < p->n_bands; bnd++) {
            // sorted by signed x separation (negated for mirrored items): the grid column
            // +-dx nu / (c du) + M/2 is then non-decreasing along the list for every channel
            auto key = [&](int it) { return (it & 1) ? -dxy[it >> 1].x : dxy[it >> 1].x; };
            std::stable_sort(bins[bnd].begin(), bins[bnd].end(), [&](int a, int b) { return key(a) < key(b); });
            band_items.insert(band_items.end(), bins[bnd].begin(), bins[bnd].end());
            band_off.push_back((int)band_items.size());
        }
        p->n_band_items = (int)band_items.size();
        // 1 / Fourier transform of the ES kernel at image column x, frequency (x - n/2)/M cycles
        // per cell: Phi(f) = 4 int_{-1}^{1} phi(z) cos(8 pi z f) dz.
        std::vector<double> gx, gw;
        gauss_legendre(200, gx, gw);
        const double beta = 2.30 * 8.0;
        corr.resize(n_pix);
        for (int x = 0; x < n_pix; x++) {
            const double f = (double)(x - n_pix / 2) / (double)M;
            double s = 0.0;
            for (size_t q = 0; q < gx.size(); q++) {
                const double z = gx[q];
                s += gw[q] * exp(beta * (sqrt(1.0 - z * z) - 1.0)) * cos(8.0 * M_PI * z * f);
            }
            corr[x] = (float)(1.0 / (4.0 * s));
        }
    }

    auto up = [&](void **dst, const void *src, size_t bytes) -> bool {
        if (bytes == 0) bytes = 16;
        if (hipMalloc(dst, bytes) != hipSuccess) return false;
        return src ? hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess : true;
    };
    bool ok = up((void **)&p->d_xyz, ant_xyz_host, sizeof(double) * 3 * n_ant) &&
              up((void **)&p->d_freq, freq_hz_host, sizeof(double) * n_chan) &&
              up((void **)&p->d_nb, nullptr, sizeof(int) * n_chan) &&
              up((void **)&p->d_pairs, pairs.data(), sizeof(int2) * pairs.size()) &&
              up((void **)&p->d_dxy, dxy.data(), sizeof(double2) * dxy.size());
    if (ok && method == NBSI_IMAGE_GRID)
        ok = up((void **)&p->d_band_off, band_off.data(), sizeof(int) * band_off.size()) &&
             up((void **)&p->d_band_items, band_items.data(), sizeof(int) * band_items.size()) &&
             up((void **)&p->d_corr, corr.data(), sizeof(float) * corr.size()) &&
             up((void **)&p->d_tmask, tmask.data(), sizeof(unsigned long long) * tmask.size()) &&
             up((void **)&p->d_tbase, tbase.data(), sizeof(int) * tbase.size()) &&
             up((void **)&p->d_inb, nullptr, sizeof(unsigned) * (size_t)n_chan * ((p->n_pairs + 31) / 32));
    if (!ok) {
        nbsi_image_plan_destroy(p);
        return nbsi_fail(ctx, NBSI_ENOMEM, "nbsi_image_plan_create: device allocation failed");
    }
    hipError_t e = launch_image_count(p, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        nbsi_image_plan_destroy(p);
        return nbsi_fail(ctx, NBSI_EHIP, std::string("nbsi_image_plan_create: ") + hipGetErrorString(e));
    }
    *out = p;
    return NBSI_OK;
}

extern "C" {

int nbsi_image_plan_create(nbsi_ctx *ctx, const double *ant_xyz_host, int n_ant, const double *freq_hz_host,
                           int n_chan, int n_pix, int method, double uv_min, double uv_max,
                           nbsi_image_plan **out) {
    return image_plan_build(ctx, ant_xyz_host, n_ant, freq_hz_host, n_chan, n_pix, method, uv_min, uv_max, 16, out);
}

int nbsi_image_plan_destroy(nbsi_image_plan *p) {
    if (!p) return NBSI_EINVAL;
    DeviceGuard g(p->device);
    void *bufs[] = {p->d_xyz,      p->d_freq,       p->d_nb,   p->d_pairs, p->d_dxy,  p->d_band_off,
                    p->d_band_items, p->d_corr, p->d_inb, p->d_tmask, p->d_tbase};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    delete p;
    return NBSI_OK;
}

int nbsi_image_plan_nbase(nbsi_image_plan *p, int64_t *n_b_host) {
    if (!p || !n_b_host) return NBSI_EINVAL;
    DeviceGuard g(p->device);
    std::vector<int> nb(p->n_chan);
    if (hipMemcpy(nb.data(), p->d_nb, sizeof(int) * p->n_chan, hipMemcpyDeviceToHost) != hipSuccess) return NBSI_EHIP;
    for (int c = 0; c < p->n_chan; c++) n_b_host[c] = nb[c];
    return NBSI_OK;
}

int nbsi_image_plan_pairs(const nbsi_image_plan *p, int *n_pairs_host, int32_t *pairs_host) {
    if (!p || !n_pairs_host) return NBSI_EINVAL;
    *n_pairs_host = p->n_pairs;
    if (pairs_host && p->n_pairs > 0) {
        DeviceGuard g(p->device);
        if (hipMemcpy(pairs_host, p->d_pairs, sizeof(int2) * p->n_pairs, hipMemcpyDeviceToHost) != hipSuccess)
            return NBSI_EHIP;
    }
    return NBSI_OK;
}

int nbsi_image(nbsi_ctx *ctx, const nbsi_image_plan *plan, const void *vis, int vis_dtype, int precision,
               float *img) {
    if (!ctx) return NBSI_EINVAL;
    if (!plan || !vis || !img) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_image: null pointer");
    if (plan->device != ctx->device) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_image: plan built on another device");
    if (vis_dtype != NBSI_VIS_I32 && vis_dtype != NBSI_VIS_F32) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_image: bad vis_dtype");
    if (precision != NBSI_PREC_FP32 && precision != NBSI_PREC_FP16 && precision != NBSI_PREC_BF16)
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_image: bad precision");
    if (!aligned16(vis) || !aligned16(img)) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_image: misaligned pointer");
    DeviceGuard g(ctx->device);
    if (plan->method == NBSI_IMAGE_DFT) {
        NBSI_TRY_HIP(ctx, launch_image_dft(plan, vis, vis_dtype, img, ctx->stream, ctx->d_flags));
        return NBSI_OK;
    }
    // Gridding runs over chunks of channels small enough for the row-transformed intermediate
    // (n_pix x n_pix complex per channel) to stay in the 256 MB last-level cache between the
    // row and column passes.
    const size_t per_chan = (size_t)plan->n_pix * plan->n_pix * sizeof(float2);
    const int chunk = (int)std::max<size_t>(1, std::min<size_t>(plan->n_chan, IMAGE_CHUNK_BYTES / per_chan));
    void *inter = nullptr, *cvis = nullptr;
    int rc = nbsi_scratch(ctx, SLOT_IMG_INTER, per_chan * chunk, &inter);
    if (rc) return rc;
    if ((rc = nbsi_scratch(ctx, SLOT_IMG_BL, sizeof(float2) * (size_t)chunk * std::max(1, plan->n_pairs), &cvis)))
        return rc;
    const size_t nprod = (size_t)(2 * plan->n_ant) * (2 * plan->n_ant + 1) / 2;
    const size_t vis_chan_bytes = nprod * 8;  // int2 or float2
    for (int c0 = 0; c0 < plan->n_chan; c0 += chunk) {
        nbsi_image_plan sub = *plan;
        sub.n_chan = std::min(chunk, plan->n_chan - c0);
        sub.d_freq = plan->d_freq + c0;
        sub.d_nb = plan->d_nb + c0;
        if (plan->d_inb) sub.d_inb = plan->d_inb + (size_t)c0 * ((plan->n_pairs + 31) >> 5);
        NBSI_TRY_HIP(ctx, launch_image_grid(&sub, (const char *)vis + vis_chan_bytes * c0, vis_dtype, precision,
                                            (float2 *)cvis, (float2 *)inter,
                                            img + (size_t)c0 * plan->n_pix * plan->n_pix, ctx->stream, ctx->d_flags));
    }
    return NBSI_OK;
}

int nbsi_image_stokes(nbsi_ctx *ctx, const nbsi_image_plan *plan, const float *stokes_i, int precision, float *img) {
    if (!ctx) return NBSI_EINVAL;
    if (!plan || !stokes_i || !img) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_image_stokes: null pointer");
    int rc = check_image_stokes(ctx, plan, precision, "nbsi_image_stokes");
    if (rc) return rc;
    if (!aligned16(stokes_i) || !aligned16(img)) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_image_stokes: misaligned pointer");
    DeviceGuard g(ctx->device);
    void *inter = nullptr;
    if ((rc = nbsi_scratch(ctx, SLOT_IMG_INTER, image_stokes_chunk(plan) * image_stokes_per_chan(plan), &inter)))
        return rc;
    NBSI_TRY_HIP(ctx, image_stokes_range(plan, stokes_i, precision, (float2 *)inter, img, 0, plan->n_chan, ctx->stream,
                                         ctx->d_flags));
    return NBSI_OK;
}

int nbsi_correlate_image(nbsi_ctx *ctx, const int8_t *spec_q, int n_chan, int n_in, int n_spec,
                         const nbsi_image_plan *plan, int precision, int n_stages, int32_t *vis, float *stokes_i,
                         float *img) {
    if (!ctx) return NBSI_EINVAL;
    int rc = nbsi_check_correlate(n_chan, n_in, n_spec);
    if (rc) return nbsi_fail(ctx, rc, "nbsi_correlate_image: bad shape");
    if (!spec_q || !vis || !plan || !stokes_i || !img) return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_correlate_image: null pointer");
    if (!aligned16(spec_q) || !aligned16(vis) || !aligned16(stokes_i) || !aligned16(img))
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_correlate_image: misaligned pointer");
    if ((rc = check_image_stokes(ctx, plan, precision, "nbsi_correlate_image"))) return rc;
    if (n_in != 2 * plan->n_ant || n_chan != plan->n_chan)
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_correlate_image: plan must be a gridding plan of n_in / 2 antennas and n_chan channels");
    if (n_stages < 0 || n_stages > NBSI_MAX_STAGES)
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_correlate_image: n_stages must be 0 .. NBSI_MAX_STAGES");
    DeviceGuard g(ctx->device);
    // Stages are whole imaging chunks, so every image is made by exactly the launches of
    // nbsi_image_stokes and the result is bit-identical to the two calls in sequence.
    const int chunk = image_stokes_chunk(plan);
    const int n_chunks = (n_chan + chunk - 1) / chunk;
    const int want = n_stages ? n_stages : NBSI_DEFAULT_STAGES;
    const int per_stage = (n_chunks + want - 1) / want * chunk;
    const int n_st = (n_chan + per_stage - 1) / per_stage;
    void *inter = nullptr, *pad = nullptr;
    if ((rc = nbsi_scratch(ctx, SLOT_IMG_INTER, chunk * image_stokes_per_chan(plan), &inter))) return rc;
    if (const size_t pb = correlate_pad_bytes(std::min(per_stage, n_chan), n_in, n_spec))
        if ((rc = nbsi_scratch(ctx, SLOT_CORR_PAD, pb, &pad))) return rc;
    if ((rc = nbsi_aux_stream(ctx))) return rc;
    const size_t q_row = (size_t)n_in * 2 * n_spec;
    const size_t v_row = (size_t)n_in * (n_in + 1);  // int32 words of one channel's visibilities
    const size_t s_row = (size_t)plan->n_pairs * 2;
    hipError_t e = hipSuccess;
    // Stage k is correlated on the caller's stream while stage k - 1 is imaged on the auxiliary
    // stream: the correlator is bound by its writes, the gridder by vector and LDS work.
    for (int k = 0; k < n_st && e == hipSuccess; k++) {
        const int c0 = k * per_stage, cn = std::min(per_stage, n_chan - c0);
        StokesOut so;
        so.mask = plan->d_tmask;
        so.base = plan->d_tbase;
        so.out = reinterpret_cast<float2 *>(stokes_i + (size_t)c0 * s_row);
        so.n_pairs = plan->n_pairs;
        e = launch_correlate_i8(spec_q + (size_t)c0 * q_row, cn, n_in, n_spec, vis + (size_t)c0 * v_row, ctx->stream, so,
                                (int8_t *)pad);
        if (e == hipSuccess) e = hipEventRecord(ctx->ev_stage[k], ctx->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(ctx->aux, ctx->ev_stage[k], 0);
        if (e == hipSuccess)
            e = image_stokes_range(plan, stokes_i, precision, (float2 *)inter, img, c0, c0 + cn, ctx->aux, ctx->d_flags);
    }
    // the caller's stream resumes only after the last image, also after a failed launch
    const hipError_t e2 = hipEventRecord(ctx->ev_stage[NBSI_MAX_STAGES], ctx->aux);
    const hipError_t e3 = e2 == hipSuccess ? hipStreamWaitEvent(ctx->stream, ctx->ev_stage[NBSI_MAX_STAGES], 0) : e2;
    if (e == hipSuccess) e = e3;
    if (e != hipSuccess) return nbsi_fail(ctx, NBSI_EHIP, std::string("nbsi_correlate_image: ") + hipGetErrorString(e));
    return NBSI_OK;
}

int nbsi_detect(nbsi_ctx *ctx, const float *img, int n_chan, int n_pix, int mode, float thresh, float *snr,
                nbsi_cand *out, int max_out, int *n_out) {
    return detect_run(ctx, img, n_chan, n_pix, mode, thresh, snr, out, max_out, n_out, nullptr, "nbsi_detect");
}

int nbsi_detect_noalloc(nbsi_ctx *ctx, const float *img, int n_chan, int n_pix, int mode, float thresh, float *snr,
                        nbsi_cand *out, int max_out, int *n_out) {
    if (!ctx) return NBSI_EINVAL;
    char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (ctx->device >= 0 && ctx->device < NBSI_MAX_DEVICES) base = static_cast<char *>(g_scratch_ptr[ctx->device]);
    }
    if (!base) return nbsi_fail(ctx, NBSI_EHIP, "nbsi_detect_noalloc: the device's fixed workspace was not resolved");
    DetectWs ws;
    ws.counter = reinterpret_cast<int *>(base + NOALLOC_OFF_COUNTER);
    ws.stats = reinterpret_cast<float *>(base + NOALLOC_OFF_STATS);
    ws.cand = reinterpret_cast<nbsi_cand *>(base + NOALLOC_OFF_CAND);
    ws.keys = reinterpret_cast<unsigned long long *>(base + NOALLOC_OFF_KEYS);
    ws.cap = NBSI_DETECT_NOALLOC_MAX_CANDS;
    return detect_run(ctx, img, n_chan, n_pix, mode, thresh, snr, out, max_out, n_out, &ws, "nbsi_detect_noalloc");
}

}  // extern "C"
