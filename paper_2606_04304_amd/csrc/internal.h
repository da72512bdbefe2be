// Internal declarations shared by the host API and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "nbsi.h"

struct nbsi_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string last_error;
    // grow-only scratch slots, each owned by one stage
    void *scratch[16] = {nullptr};
    size_t scratch_size[16] = {0};
    int *d_counter = nullptr;  // small device counters (detector)
    unsigned *d_flags = nullptr;  // NBSI_FLAG_* bits set by kernels, read and cleared by nbsi_status
    // auxiliary stream and events of the overlapped correlate + image call (created on first use)
    hipStream_t aux = nullptr;
    hipEvent_t ev_stage[NBSI_MAX_STAGES + 1] = {};
    // orders the work of a new stream after the context's earlier work (nbsi_set_stream), so
    // calls on several streams never overlap on the context's scratch
    hipEvent_t ev_switch = nullptr;
};

enum ScratchSlot {
    SLOT_CHAN_STAGE_Q = 0,  // channelizer staging, int8
    SLOT_CHAN_STAGE_F = 1,  // channelizer staging, float32
    SLOT_IMG_INTER = 2,     // imager: row-transformed grid
    SLOT_DET_CAND = 3,      // detector: unsorted candidates
    SLOT_DET_KEYS = 4,      // detector: sort keys
    SLOT_DET_STATS = 5,     // detector: per-channel / per-pixel statistics
    SLOT_IMG_BL = 6,        // imager: per-channel baseline values
    SLOT_CORR_PAD = 7,      // correlator: spectra repacked to a 16-byte row stride
    SLOT_SEARCH_S = 8,      // search: best matched-filter SNR per voxel
    SLOT_SEARCH_W = 9,      // search: its width per voxel
    SLOT_SEARCH_HIST = 10,  // search: SNR histogram
    SLOT_SEARCH_VALS = 11,  // search: exact SNRs of one histogram bin
    SLOT_SEARCH_CAND = 12,  // search: provisional detections
    SLOT_SEARCH_KEEP = 13,  // search: their keep flags
    SLOT_SEARCH_SURV = 14,  // search: survivors of the suppression
    SLOT_S2_PSF = 15,       // Stage II: unit visibilities and point-spread-function images
};


struct nbsi_image_plan {
    int device = 0;
    int n_ant = 0, n_chan = 0, n_pix = 0, method = 0;
    double uv_min = 0, uv_max = 0;
    // device arrays
    double *d_xyz = nullptr;      // [n_ant][3]
    double *d_freq = nullptr;     // [n_chan]
    int *d_nb = nullptr;          // [n_chan] |B| per channel
    int2 *d_pairs = nullptr;      // candidate pairs (a, b), a > b
    double2 *d_dxy = nullptr;     // (x_a - x_b, y_a - y_b) metres of each candidate pair
    int n_pairs = 0;
    // gridding: candidate pairs binned by bands of the grid rows v >= 0 (array rows n_pix ..
    // 2 n_pix - 1; CSR over bands); a workgroup holds 256 * ge grid cells (ge = 16 or 32), i.e.
    // band_rows = 256 ge / (2 n_pix) rows, and n_bands = n_pix / band_rows
    int ge = 16, band_rows = 0, n_bands = 0;
    int *d_band_off = nullptr;    // [n_bands + 1]
    int *d_band_items = nullptr;  // 2 * (index into d_pairs) + 1 if gridded at -(u, v) with conj V
    int n_band_items = 0;
    float *d_corr = nullptr;      // [n_pix] 1 / (kernel Fourier transform) per image column
    // gridding plans: membership bitmap of B, [n_chan][(n_pairs + 31) / 32] words (bit k % 32 of
    // word k / 32 = pair k imaged at that channel), written by the count kernel
    unsigned *d_inb = nullptr;
    // Candidates are ordered by 8 x 8 antenna block (a / 8, b / 8), blocks in packed lower-triangle
    // order, then by (a % 8) * 8 + b % 8 within a block: block t holds the pairs whose bits are set
    // in d_tmask[t], numbered from d_tbase[t] (gridding plans)
    unsigned long long *d_tmask = nullptr;
    int *d_tbase = nullptr;
};

// Makes dev current for the scope (restoring the caller's device on exit).
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

#define NBSI_TRY_HIP(ctx, call)                                                        \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            (ctx)->last_error = std::string(#call) + ": " + hipGetErrorString(e_);    \
            return NBSI_EHIP;                                                          \
        }                                                                              \
    } while (0)

int nbsi_scratch(nbsi_ctx *ctx, int slot, size_t bytes, void **ptr);

// Channels of a gridded image are processed in chunks whose row-pass intermediate (n_pix x n_pix
// complex float per channel) stays within this many bytes, so the column pass reads it from the
// 256 MB last-level cache rather than from HBM.
constexpr size_t IMAGE_CHUNK_BYTES = (size_t)128 << 20;
int image_plan_build(nbsi_ctx *ctx, const double *ant_xyz_host, int n_ant, const double *freq_hz_host, int n_chan,
                     int n_pix, int method, double uv_min, double uv_max, int ge, nbsi_image_plan **out);
int nbsi_fail(nbsi_ctx *ctx, int code, const std::string &msg);

// Batched launches: every stage of several sub-bands runs as one launch over a task table,
// one workgroup per task; each job (sub-band, or channel range of one) records the first task
// it owns, and a workgroup finds its job by a scan of the (few) jobs.

// One sub-band's channelizer parameters (device-visible; also the job of a batched launch).
struct ChanJob {
    const int8_t *volt;
    const float *gain;
    int8_t *stage_q;
    float2 *stage_f;
    int log_n, n_spec, klo, n_chan;
    int task0;  // first task of this sub-band in a batched launch
    unsigned *flags;  // NBSI_FLAG_* bits (null: not reported)
};

// One sub-band's correlator parameters (the job of a batched launch).
struct CorrJob {
    const int8_t *q;
    int32_t *vis;
    int n_in, n_spec, n_chan;
    int task0;
};
enum { CORR_VARIANT_TILED = 0, CORR_VARIANT_CHAN32 = 1, CORR_VARIANT_CHAN64 = 2 };
int correlate_batch_tasks(const CorrJob &jb, int variant);
int correlate_default_variant(int n_in, int n_spec);
// Tiled correlations of at least this many spectra take 256 x 256 tiles, the rest (at most 64
// spectra: whole-channel shapes too large for LDS) 128 x 128 tiles.  (Measured at 704 inputs:
// the 256 tiles are faster from T = 80 on, 0.50 vs 0.71 ms at T = 80 and 1.04 vs 1.34 at 298.)
constexpr int PIPE_BIG_T = 65;
bool correlate_variant_valid(int n_in, int n_spec, int variant);
// Optional Stokes-I output of the correlator's epilogue: for the candidate pair (A, B) of an
// imaging plan with index k (see nbsi_image_plan::d_tmask), out[c * n_pairs + k] =
// (V_XX + V_YY) / 2 of channel c, computed exactly as the imager's gather computes it (inputs
// 2A, 2A + 1 are antenna A's two polarisations).
struct StokesOut {
    const unsigned long long *mask = nullptr;
    const int *base = nullptr;
    float2 *out = nullptr;
    int n_pairs = 0;
};
// pad_scratch (correlate_pad_bytes bytes, or null for the byte-load fallback) receives the
// spectra repacked to a 16-byte row stride when the tiled variant gets n_spec % 16 != 0.
// calw (optional, [n_chan][n_in] complex float): write w_i V_ij conj(w_j) as float32 instead of
// the int32 visibilities.
hipError_t launch_correlate_variant(const int8_t *q, int n_chan, int n_in, int n_spec, int32_t *vis, int variant,
                                    hipStream_t st, StokesOut so = StokesOut(), int8_t *pad_scratch = nullptr,
                                    const float2 *calw = nullptr);
size_t correlate_pad_bytes(int n_chan, int n_in, int n_spec);
// vec: every job's n_spec is a multiple of 16 (the tiled variant then stages whole vectors)
hipError_t launch_correlate_batch(const CorrJob *d_jobs, int n_jobs, int n_tasks, int variant, int n_in, bool vec,
                                  hipStream_t st);

// One sub-band's (or channel range's) gridding imager parameters (the job of batched launches).
struct ImgJob {
    const int32_t *vis;
    const double *xyz, *freq;
    const int2 *pairs;
    const double2 *dxy;
    const int *band_off, *band_items, *nb;
    const unsigned *inb;  // membership bitmap rows from the job's first channel
    const float *corr;
    float2 *cvis, *inter;
    float *img;
    int n_pairs, n_ant, n_pix, log_m, n_bands, n_chan;
    double uv_min, uv_max;
    int gather_task0, rows_task0, cols_task0;
    unsigned *flags = nullptr;  // NBSI_FLAG_* bits (null: not reported)
};
// Image columns per workgroup of the gridding imager's column pass: a tile of 256 ge cells
// holds 256 ge / n_pix columns of n_pix complex values, at most the n_pix columns there are.
__host__ __device__ constexpr int cols_per_band(int ge, int n_pix) {
    return 256 * ge / n_pix < n_pix ? 256 * ge / n_pix : n_pix;
}

hipError_t launch_image_batch_gather(const ImgJob *d_jobs, int n_jobs, int n_tasks, hipStream_t st);
hipError_t launch_image_batch_rows(const ImgJob *d_jobs, int n_jobs, int n_tasks, int log_m, int precision, int ge,
                                   hipStream_t st);
hipError_t launch_image_batch_cols(const ImgJob *d_jobs, int n_jobs, int n_tasks, int log_m, int ge, hipStream_t st);

int channelize_log_m(int log_n, int n_chan);
int channelize_dyn_elems(int log_n, int log_m);
int channelize_group(int log_n, int log_m);
int corner_turn_tasks(int n_in, int n_spec, int n_chan);
hipError_t launch_corner_turn_q_batch(const ChanJob *d_jobs, int n_jobs, const int *d_task0, int n_tasks,
                                      int8_t *const *d_outs, int n_in, hipStream_t st);

// ---- launchers (each returns hipError_t of the launch) ----
hipError_t launch_channelize(const int8_t *volt, int n_in, int log_n, int n_spec, int klo,
                             int n_chan, const float *gain, int8_t *stage_q, float *stage_f,
                             hipStream_t st, unsigned *flags = nullptr);
hipError_t launch_channelize_batch(const ChanJob *d_jobs, int n_jobs, int n_tasks, int log_m, int g,
                                   int max_dyn_elems, hipStream_t st);
hipError_t launch_corner_turn_q(const int8_t *stage, int n_in, int n_spec, int n_chan,
                                int8_t *out, hipStream_t st);
hipError_t launch_corner_turn_f(const float *stage, int n_in, int n_spec, int n_chan, float *out,
                                hipStream_t st);
hipError_t launch_correlate_i8(const int8_t *q, int n_chan, int n_in, int n_spec, int32_t *vis,
                               hipStream_t st, StokesOut so = StokesOut(), int8_t *pad_scratch = nullptr,
                               const float2 *calw = nullptr);
hipError_t launch_correlate_f32(const float *q, int n_chan, int n_in, int n_spec, float *vis,
                                hipStream_t st);
hipError_t launch_image_count(const nbsi_image_plan *p, hipStream_t st);
hipError_t launch_image_dft(const nbsi_image_plan *p, const void *vis, int vis_dtype, float *img,
                            hipStream_t st, unsigned *flags = nullptr);
hipError_t launch_image_grid(const nbsi_image_plan *p, const void *vis, int vis_dtype,
                             int precision, float2 *cvis, float2 *inter, float *img, hipStream_t st,
                             unsigned *flags = nullptr);
hipError_t launch_image_grid_stokes(const nbsi_image_plan *p, const float2 *cvis, int precision, float2 *inter,
                                    float *img, hipStream_t st, unsigned *flags = nullptr);
hipError_t launch_detect_stats(const float *img, int n_chan, int n_pix, int mode, float *stats,
                               hipStream_t st);
hipError_t launch_detect_scan(const float *img, int n_chan, int n_pix, int mode,
                              const float *stats, float thresh, float *snr, nbsi_cand *cand,
                              int cap, int *counter, hipStream_t st, unsigned *flags = nullptr);
// Sorts the candidates on the device when their count (read there) is at most
// detect_sort_small_max() and at most cap; larger counts are left to launch_detect_sort.
hipError_t launch_detect_sort_small_dev(const nbsi_cand *cand, const int *counter, int cap, int n_chan, int n_pix,
                                       nbsi_cand *out, int n_out, hipStream_t st);
int detect_sort_small_max();
hipError_t launch_detect_sort(nbsi_cand *cand, int n, unsigned long long *keys, int n_chan,
                              int n_pix, nbsi_cand *out, int n_out, hipStream_t st);
