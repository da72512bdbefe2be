// Batched execution of uneven sub-bands (the paper's batch-by-batch processing of the band,
// Sec. 2.1, with variable FFT lengths and integrations as in its follow-up, Sec. 2.6):
// channelize -> corner turn -> correlate -> image for every sub-band, each stage one launch
// over a task table spanning the sub-bands (grouped only where kernel shapes differ; the
// imager per cache-sized chunk of channels), one workgroup per task, the whole sequence
// captured once into a hipGraph and replayed.  A persistent form with a device work queue was
// measured slower here: the tasks are small and uneven, and the hardware dispatcher spreads
// them better than an atomic counter per task.
// An autotuner chooses the correlator variant (tiles or whole-channel panels) per integration
// length and the gridding tile height (16 or 32 cells per thread) per image shape by timing
// replays of the whole batch, and caches the choices in a text file.  Tiled sub-bands whose rows
// are whole 16-byte vectors take the single-band persistent kernel, one launch per sub-band (each
// fills the GPU); the others the batched tiled kernel.
#include "internal.h"

#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

int correlate_batch_tasks(const CorrJob &jb, int variant);
hipError_t correlate_batch_prepare(int variant, int n_in);

struct nbsi_batch {
    nbsi_ctx *ctx = nullptr;
    int device = 0, n_sb = 0, n_ant = 0, n_in = 0, precision = 0, flags = 0;
    std::vector<nbsi_subband> sb;
    std::vector<nbsi_image_plan *> plans;
    std::vector<int> corr_variant, grid_ge;
    std::vector<void *> owned;  // device allocations of the batch
    std::vector<int8_t *> stage;
    float2 *cvis = nullptr;        // one imaging chunk's Stokes-I gather
    float2 *inter = nullptr;       // one imaging chunk's row-pass intermediate
    size_t cvis_bytes = 0, inter_bytes = 0;

    struct Launch {  // one batched launch: kind, shape key, job array on the device
        // 0 channelize, 1 corner turn, 2 correlate, 3 gather, 4 rows, 5 cols, 6 correlate with the
        // single-band tiled kernel once per job (h_corr)
        int kind;
        int a = 0, b = 0;  // kind-specific shape (log_m/g, variant, log_m/ge)
        int group = 0;     // sub-band group (one group per sub-band with NBSI_BATCH_OVERLAP)
        int n_jobs = 0, n_tasks = 0, max_dyn = 0;
        void *d_jobs = nullptr;
        int *d_task0 = nullptr;
        int8_t **d_outs = nullptr;
        std::vector<CorrJob> h_corr;
    };
    std::vector<Launch> launches;

    hipStream_t stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // NBSI_BATCH_OVERLAP: correlate and image launches run on `aux`, each group after the event
    // recorded behind its corner turn on `stream`; `stream` joins `aux` at the end
    hipStream_t aux = nullptr;
    std::vector<hipEvent_t> ev_grp;
    hipEvent_t ev_join = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool captured = false;
    std::string desc;
};

namespace {

template <typename T>
int upload(nbsi_batch *b, const std::vector<T> &v, T **out) {
    void *p = nullptr;
    if (hipMalloc(&p, sizeof(T) * std::max<size_t>(1, v.size())) != hipSuccess) return NBSI_ENOMEM;
    b->owned.push_back(p);
    if (!v.empty() && hipMemcpy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess)
        return NBSI_EHIP;
    *out = (T *)p;
    return NBSI_OK;
}

int alloc(nbsi_batch *b, size_t bytes, void **out) {
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(256, bytes)) != hipSuccess) return NBSI_ENOMEM;
    b->owned.push_back(p);
    *out = p;
    return NBSI_OK;
}

// ---- tuning cache: one "key value" pair per line ----
std::map<std::string, int> read_cache(const char *path) {
    std::map<std::string, int> m;
    if (!path) return m;
    FILE *f = fopen(path, "r");
    if (!f) return m;
    char key[256];
    int val;
    while (fscanf(f, "%255s %d", key, &val) == 2) m[key] = val;
    fclose(f);
    return m;
}

void write_cache(const char *path, const std::map<std::string, int> &m) {
    if (!path) return;
    FILE *f = fopen(path, "w");
    if (!f) return;
    for (auto &kv : m) fprintf(f, "%s %d\n", kv.first.c_str(), kv.second);
    fclose(f);
}

std::string corr_key(int n_in, int n_spec) {
    return "corr_n_in=" + std::to_string(n_in) + ",n_spec=" + std::to_string(n_spec);
}
std::string grid_key(int n_ant, int n_pix, int n_chan) {
    return "grid_n_ant=" + std::to_string(n_ant) + ",n_pix=" + std::to_string(n_pix) + ",n_chan=" +
           std::to_string(n_chan);
}

double time_ms(hipStream_t st, const std::function<hipError_t()> &fn, int reps) {
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    if (fn() != hipSuccess) return 1e30;  // warm-up
    (void)hipEventRecord(a, st);
    for (int r = 0; r < reps; r++)
        if (fn() != hipSuccess) return 1e30;
    (void)hipEventRecord(b, st);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / reps;
}

// Every stage of every sub-band, as the grouped launches.
hipError_t launch_one(const nbsi_batch *b, const nbsi_batch::Launch &L, hipStream_t st) {
    switch (L.kind) {
        case 0: return launch_channelize_batch((const ChanJob *)L.d_jobs, L.n_jobs, L.n_tasks, L.a, L.b, L.max_dyn, st);
        case 1:
            return launch_corner_turn_q_batch((const ChanJob *)L.d_jobs, L.n_jobs, L.d_task0, L.n_tasks, L.d_outs,
                                              b->n_in, st);
        case 2: return launch_correlate_batch((const CorrJob *)L.d_jobs, L.n_jobs, L.n_tasks, L.a, b->n_in, L.b != 0, st);
        case 3: return launch_image_batch_gather((const ImgJob *)L.d_jobs, L.n_jobs, L.n_tasks, st);
        case 4: return launch_image_batch_rows((const ImgJob *)L.d_jobs, L.n_jobs, L.n_tasks, L.a, b->precision, L.b, st);
        case 5: return launch_image_batch_cols((const ImgJob *)L.d_jobs, L.n_jobs, L.n_tasks, L.a, L.b, st);
        case 6:
            for (const CorrJob &j : L.h_corr) {
                const hipError_t e = launch_correlate_variant(j.q, j.n_chan, j.n_in, j.n_spec, j.vis, CORR_VARIANT_TILED,
                                                              st, StokesOut(), nullptr, nullptr);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
    }
    return hipErrorInvalidValue;
}

hipError_t enqueue_all(nbsi_batch *b, hipStream_t st) {
    if (!b->aux) {
        for (const auto &L : b->launches) {
            const hipError_t e = launch_one(b, L, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    // overlapped: channelize + corner turn of every group in order on st; a group's correlate
    // and image launches on aux once its corner turn is done, so group g + 1 is channelized
    // while group g is correlated and imaged
    int last_linked = -1;
    for (const auto &L : b->launches) {
        const bool back = L.kind >= 2;
        if (back && L.group != last_linked) {
            hipError_t e = hipEventRecord(b->ev_grp[L.group], st);
            if (e == hipSuccess) e = hipStreamWaitEvent(b->aux, b->ev_grp[L.group], 0);
            if (e != hipSuccess) return e;
            last_linked = L.group;
        }
        const hipError_t e = launch_one(b, L, back ? b->aux : st);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipEventRecord(b->ev_join, b->aux);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, b->ev_join, 0);
    return e;
}

// The launches of the sub-bands `members` (in order), tagged with `group`.
int build_group_launches(nbsi_batch *b, const std::vector<int> &members, int group) {
    const size_t first = b->launches.size();
    // channelize: one launch per (sub-transform size, load grouping, FFT length): the table LDS is
    // sized by the FFT length, and one size per launch keeps the occupancy of the shorter ones
    std::map<std::tuple<int, int, int>, std::vector<int>> cg;
    for (int s : members) {
        const int log_n = 31 - __builtin_clz(b->sb[s].n_fft);
        const int lm = channelize_log_m(log_n, b->sb[s].n_chan);
        cg[std::make_tuple(lm, channelize_group(log_n, lm), log_n)].push_back(s);
    }
    for (auto &kv : cg) {
        std::vector<ChanJob> jobs;
        int tasks = 0, max_dyn = 0;
        for (int s : kv.second) {
            const nbsi_subband &x = b->sb[s];
            const int log_n = 31 - __builtin_clz(x.n_fft);
            ChanJob j{x.volt, x.gain, b->stage[s], nullptr, log_n, x.n_spec, (x.chan0 + x.n_fft / 2) & (x.n_fft - 1),
                      x.n_chan, tasks, b->ctx->d_flags};
            jobs.push_back(j);
            tasks += b->n_in * x.n_spec;
            max_dyn = std::max(max_dyn, channelize_dyn_elems(log_n, std::get<0>(kv.first)));
        }
        nbsi_batch::Launch L;
        L.kind = 0;
        L.a = std::get<0>(kv.first);
        L.b = std::get<1>(kv.first);
        L.n_jobs = (int)jobs.size();
        L.n_tasks = tasks;
        L.max_dyn = max_dyn;
        int rc = upload(b, jobs, (ChanJob **)&L.d_jobs);
        if (rc) return rc;
        b->launches.push_back(L);
    }
    // corner turn: one launch over every sub-band
    {
        std::vector<ChanJob> jobs;
        std::vector<int> t0;
        std::vector<int8_t *> outs;
        int tasks = 0;
        for (int s : members) {
            const nbsi_subband &x = b->sb[s];
            jobs.push_back(ChanJob{x.volt, x.gain, b->stage[s], nullptr, 0, x.n_spec, 0, x.n_chan, tasks});
            t0.push_back(tasks);
            outs.push_back(x.spec_q);
            tasks += corner_turn_tasks(b->n_in, x.n_spec, x.n_chan);
        }
        nbsi_batch::Launch L;
        L.kind = 1;
        L.n_jobs = (int)members.size();
        L.n_tasks = tasks;
        int rc = upload(b, jobs, (ChanJob **)&L.d_jobs);
        if (!rc) rc = upload(b, t0, &L.d_task0);
        if (!rc) rc = upload(b, outs, &L.d_outs);
        if (rc) return rc;
        b->launches.push_back(L);
    }
    // correlate: group by variant (and, for the tiled variant, by whether the spectra rows are
    // whole 16-byte vectors, which selects the vector-load form of its staging)
    std::map<std::pair<int, int>, std::vector<int>> kg;
    for (int s : members) {
        const int v = b->corr_variant[s];
        kg[{v, v == CORR_VARIANT_TILED && (b->sb[s].n_spec & 15) == 0 ? 1 : 0}].push_back(s);
    }
    for (auto &kv : kg) {
        if (kv.first.first == CORR_VARIANT_TILED && kv.first.second) {
            // whole 16-byte rows: the persistent, pipelined single-band kernel, one launch per
            // sub-band (each fills the GPU on its own)
            nbsi_batch::Launch L;
            L.kind = 6;
            for (int s : kv.second) {
                const nbsi_subband &x = b->sb[s];
                L.h_corr.push_back(CorrJob{x.spec_q, x.vis, b->n_in, x.n_spec, x.n_chan, 0});
            }
            L.n_jobs = (int)L.h_corr.size();
            b->launches.push_back(L);
            continue;
        }
        std::vector<CorrJob> jobs;
        int tasks = 0;
        for (int s : kv.second) {
            const nbsi_subband &x = b->sb[s];
            CorrJob j{x.spec_q, x.vis, b->n_in, x.n_spec, x.n_chan, tasks};
            jobs.push_back(j);
            tasks += correlate_batch_tasks(j, kv.first.first);
        }
        hipError_t e = correlate_batch_prepare(kv.first.first, b->n_in);
        if (e != hipSuccess) return NBSI_EHIP;
        nbsi_batch::Launch L;
        L.kind = 2;
        L.a = kv.first.first;
        L.b = kv.first.second;
        L.n_jobs = (int)jobs.size();
        L.n_tasks = tasks;
        int rc = upload(b, jobs, (CorrJob **)&L.d_jobs);
        if (rc) return rc;
        b->launches.push_back(L);
    }
    // imager: per channel chunk a gather, a rows and a columns launch (below)
    std::vector<ImgJob> base(b->n_sb);
    for (int s : members) {
        const nbsi_image_plan *p = b->plans[s];
        ImgJob &j = base[s];
        j.vis = b->sb[s].vis;
        j.xyz = p->d_xyz;
        j.freq = p->d_freq;
        j.pairs = p->d_pairs;
        j.dxy = p->d_dxy;
        j.band_off = p->d_band_off;
        j.band_items = p->d_band_items;
        j.nb = p->d_nb;
        j.inb = p->d_inb;
        j.corr = p->d_corr;
        j.cvis = b->cvis;
        j.inter = b->inter;
        j.img = b->sb[s].img;
        j.n_pairs = p->n_pairs;
        j.n_ant = p->n_ant;
        j.n_pix = p->n_pix;
        j.log_m = 31 - __builtin_clz(2 * p->n_pix);
        j.n_bands = p->n_bands;
        j.n_chan = p->n_chan;
        j.uv_min = p->uv_min;
        j.uv_max = p->uv_max;
        j.flags = b->ctx->d_flags;
    }
    // channel chunks of every sub-band of one (transform size, tile height), each chunk's row
    // intermediate within IMAGE_CHUNK_BYTES: per chunk a gather, a rows and a columns launch, so
    // the Stokes-I gather and the intermediate are read back while still in the last-level cache
    std::map<std::pair<int, int>, std::vector<int>> rg;
    for (int s : members) rg[{base[s].log_m, b->grid_ge[s]}].push_back(s);
    for (auto &kv : rg) {
        const int ge = kv.first.second;
        std::vector<ImgJob> chunk;
        size_t used = 0, cv_used = 0;  // bytes of the chunk's intermediate and Stokes-I gather
        auto flush = [&]() -> int {
            if (chunk.empty()) return NBSI_OK;
            std::vector<ImgJob> gath = chunk, rows = chunk, cols = chunk;
            int gt = 0, rt = 0, ct = 0;
            for (size_t q = 0; q < chunk.size(); q++) {
                gath[q].gather_task0 = gt;
                gt += chunk[q].n_chan * ((chunk[q].n_pairs + 255) / 256);
                rows[q].rows_task0 = rt;
                rt += chunk[q].n_chan * chunk[q].n_bands;
                cols[q].cols_task0 = ct;
                ct += chunk[q].n_chan * (chunk[q].n_pix / cols_per_band(ge, chunk[q].n_pix));
            }
            nbsi_batch::Launch G;
            G.kind = 3;
            G.n_jobs = (int)gath.size();
            G.n_tasks = gt;
            int rc0 = upload(b, gath, (ImgJob **)&G.d_jobs);
            if (rc0) return rc0;
            b->launches.push_back(G);
            nbsi_batch::Launch R;
            R.kind = 4;
            R.a = kv.first.first;
            R.b = ge;
            R.n_jobs = (int)rows.size();
            R.n_tasks = rt;
            int rc = upload(b, rows, (ImgJob **)&R.d_jobs);
            if (rc) return rc;
            b->launches.push_back(R);
            nbsi_batch::Launch C;
            C.kind = 5;
            C.a = kv.first.first;
            C.b = ge;
            C.n_jobs = (int)cols.size();
            C.n_tasks = ct;
            rc = upload(b, cols, (ImgJob **)&C.d_jobs);
            if (rc) return rc;
            b->launches.push_back(C);
            chunk.clear();
            used = 0;
            cv_used = 0;
            return NBSI_OK;
        };
        for (int s : kv.second) {
            const ImgJob &j = base[s];
            const size_t per_chan = (size_t)j.n_pix * j.n_pix * sizeof(float2);
            const size_t nb = (size_t)j.n_pix * j.n_pix;
            for (int c0 = 0; c0 < j.n_chan;) {
                if (used + per_chan > IMAGE_CHUNK_BYTES && !chunk.empty()) {
                    const int rc = flush();
                    if (rc) return rc;
                }
                const int fit = (int)std::max<size_t>(1, (IMAGE_CHUNK_BYTES - std::min(used, IMAGE_CHUNK_BYTES)) / per_chan);
                const int n = std::min(j.n_chan - c0, fit);
                ImgJob q = j;  // channels [c0, c0 + n) of this sub-band, pointers moved to them
                const size_t nprod = (size_t)(2 * j.n_ant) * (2 * j.n_ant + 1) / 2;
                q.vis = j.vis + (size_t)c0 * nprod * 2;
                q.freq = j.freq + c0;
                q.nb = j.nb + c0;
                q.inb = j.inb + (size_t)c0 * ((j.n_pairs + 31) >> 5);
                const size_t cv_n = sizeof(float2) * (size_t)n * std::max(1, j.n_pairs);
                if (!b->cvis || !b->inter || used + per_chan * n > b->inter_bytes || cv_used + cv_n > b->cvis_bytes)
                    return NBSI_EINVAL;  // the chunk buffers were sized for fewer pairs or channels
                q.cvis = b->cvis + cv_used / sizeof(float2);
                q.inter = b->inter + used / sizeof(float2);
                q.img = j.img + (size_t)c0 * nb;
                q.n_chan = n;
                chunk.push_back(q);
                used += per_chan * n;
                cv_used += cv_n;
                c0 += n;
            }
        }
        const int rc = flush();
        if (rc) return rc;
    }
    for (size_t i = first; i < b->launches.size(); i++) b->launches[i].group = group;
    return NBSI_OK;
}

// Every sub-band in one group (each stage one launch over all of them, grouped by shape), or
// with NBSI_BATCH_OVERLAP one group per sub-band, so that the stages of consecutive sub-bands
// can overlap.
int build_launches(nbsi_batch *b) {
    std::vector<std::vector<int>> groups;
    if (b->flags & NBSI_BATCH_OVERLAP) {
        for (int s = 0; s < b->n_sb; s++) groups.push_back({s});
    } else {
        groups.emplace_back();
        for (int s = 0; s < b->n_sb; s++) groups.back().push_back(s);
    }
    for (size_t g = 0; g < groups.size(); g++)
        if (const int rc = build_group_launches(b, groups[g], (int)g)) return rc;
    return NBSI_OK;
}

void free_batch(nbsi_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->aux) (void)hipStreamSynchronize(b->aux);
    for (auto *p : b->plans)
        if (p) nbsi_image_plan_destroy(p);
    for (void *p : b->owned) (void)hipFree(p);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    for (hipEvent_t e : b->ev_grp)
        if (e) (void)hipEventDestroy(e);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    if (b->aux) (void)hipStreamDestroy(b->aux);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // namespace

extern "C" {

int nbsi_batch_plan(nbsi_ctx *ctx, const double *ant_xyz_host, int n_ant, const nbsi_subband *sb, int n_sb,
                    int precision, int flags, const char *tune_cache_path, nbsi_batch **out) {
    if (!ctx || !out) return NBSI_EINVAL;
    *out = nullptr;
    if (!sb || n_sb < 1 || n_sb > 4096 || !ant_xyz_host || n_ant < 2)
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_batch_plan: bad arguments");
    if (precision != NBSI_PREC_FP32 && precision != NBSI_PREC_FP16 && precision != NBSI_PREC_BF16)
        return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_batch_plan: bad precision");
    const int n_in = 2 * n_ant;
    for (int s = 0; s < n_sb; s++) {
        const nbsi_subband &x = sb[s];
        int rc = nbsi_check_channelize(n_in, x.n_fft, x.n_spec, x.chan0, x.n_chan);
        if (!rc) rc = nbsi_check_image(x.n_chan, n_ant, x.n_pix, NBSI_IMAGE_GRID, precision, 0.0, INFINITY);
        if (rc) return nbsi_fail(ctx, rc, "nbsi_batch_plan: sub-band " + std::to_string(s) + " has a bad shape");
        if (!x.volt || !x.gain || !x.freq_hz_host || !x.spec_q || !x.vis || !x.img)
            return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_batch_plan: sub-band " + std::to_string(s) + " null pointer");
        const void *ptrs[] = {x.volt, x.gain, x.spec_q, x.vis, x.img};
        for (const void *p : ptrs)
            if ((uintptr_t)p & 15u)
                return nbsi_fail(ctx, NBSI_EINVAL, "nbsi_batch_plan: sub-band " + std::to_string(s) + " misaligned");
    }
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != ctx->device) (void)hipSetDevice(ctx->device);
    nbsi_batch *b = new (std::nothrow) nbsi_batch();
    if (!b) return NBSI_ENOMEM;
    b->ctx = ctx;
    b->device = ctx->device;
    b->n_sb = n_sb;
    b->n_ant = n_ant;
    b->n_in = n_in;
    b->precision = precision;
    b->flags = flags;
    b->sb.assign(sb, sb + n_sb);
    int rc = NBSI_OK;
    auto fail = [&](int code, const std::string &msg) {
        free_batch(b);
        if (prev >= 0 && prev != ctx->device) (void)hipSetDevice(prev);
        return nbsi_fail(ctx, code, "nbsi_batch_plan: " + msg);
    };
    // a dedicated stream of default priority (graph capture cannot use the null stream)
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess)
        return fail(NBSI_EHIP, "stream/event creation failed");
    if (flags & NBSI_BATCH_OVERLAP) {
        if (hipStreamCreateWithFlags(&b->aux, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming) != hipSuccess)
            return fail(NBSI_EHIP, "stream/event creation failed");
        b->ev_grp.assign(n_sb, nullptr);
        for (int s = 0; s < n_sb; s++)
            if (hipEventCreateWithFlags(&b->ev_grp[s], hipEventDisableTiming) != hipSuccess)
                return fail(NBSI_EHIP, "stream/event creation failed");
    }
    std::map<std::string, int> cache = read_cache(tune_cache_path);
    bool cache_dirty = false;
    // per sub-band scratch, default choices
    for (int s = 0; s < n_sb; s++) {
        const nbsi_subband &x = b->sb[s];
        void *st = nullptr;
        if ((rc = alloc(b, (size_t)n_in * x.n_spec * x.n_chan * 2, &st))) return fail(rc, "out of memory");
        b->stage.push_back((int8_t *)st);
        b->corr_variant.push_back(correlate_default_variant(n_in, x.n_spec));
        b->grid_ge.push_back(16);
    }
    const bool tune = (flags & NBSI_BATCH_AUTOTUNE) != 0;
    // choices from the cache (else the defaults: correlator variant by shape, 16-cell tiles)
    for (int s = 0; s < n_sb; s++) {
        const nbsi_subband &x = b->sb[s];
        auto ic = cache.find(corr_key(n_in, x.n_spec));
        if (ic != cache.end() && correlate_variant_valid(n_in, x.n_spec, ic->second)) b->corr_variant[s] = ic->second;
        auto ig = cache.find(grid_key(n_ant, x.n_pix, x.n_chan));
        if (flags & NBSI_BATCH_GRID_TALL) b->grid_ge[s] = 32;
        else if (ig != cache.end() && (ig->second == 16 || ig->second == 32)) b->grid_ge[s] = ig->second;
    }
    auto build_plan = [&](int s, int ge, nbsi_image_plan **p) {
        const nbsi_subband &x = b->sb[s];
        return image_plan_build(ctx, ant_xyz_host, n_ant, x.freq_hz_host, x.n_chan, x.n_pix, NBSI_IMAGE_GRID, 0.0,
                                INFINITY, ge, p);
    };
    for (int s = 0; s < n_sb; s++) {
        nbsi_image_plan *p = nullptr;
        if ((rc = build_plan(s, b->grid_ge[s], &p))) return fail(rc, "plan failed");
        b->plans.push_back(p);
    }
    {
        // A chunk holds sub-bands of one transform size, so at most max(1, IMAGE_CHUNK_BYTES /
        // per-channel intermediate) channels; its gather at most that many channels times the
        // largest pair count among sub-bands of that size (pair counts do not depend on the tile
        // height, so the tuner's alternative plans fit too).
        size_t need = IMAGE_CHUNK_BYTES, cv_need = 0;
        for (int s = 0; s < n_sb; s++) {
            const size_t per_chan = (size_t)b->sb[s].n_pix * b->sb[s].n_pix * sizeof(float2);
            need = std::max(need, per_chan);
            const size_t ch = std::max<size_t>(1, IMAGE_CHUNK_BYTES / per_chan);
            size_t pairs_max = 1;
            for (int s2 = 0; s2 < n_sb; s2++)
                if (b->sb[s2].n_pix == b->sb[s].n_pix) pairs_max = std::max<size_t>(pairs_max, b->plans[s2]->n_pairs);
            cv_need = std::max(cv_need, sizeof(float2) * ch * pairs_max);
        }
        void *in = nullptr, *cv = nullptr;
        if ((rc = alloc(b, need, &in))) return fail(rc, "out of memory");
        if ((rc = alloc(b, cv_need, &cv))) return fail(rc, "out of memory");
        b->inter = (float2 *)in;
        b->cvis = (float2 *)cv;
        b->inter_bytes = need;
        b->cvis_bytes = cv_need;
    }
    if ((rc = build_launches(b))) return fail(rc, "launch tables failed");
    if (tune) {
        // Coordinate descent over shape classes, each candidate timed as a replay of the whole
        // batch (a kernel timed alone can mislead: e.g. 1,024 whole-channel correlator groups
        // leave a tail on 256 CUs that the batched launch, mixing sub-bands, does not have).
        // Shapes already in the cache keep their choice; a change is kept when the batch gets
        // more than 1% faster, so the tuned batch is never slower than the default one.
        auto relaunch = [&]() {
            b->launches.clear();
            return build_launches(b);
        };
        auto time_batch = [&]() { return time_ms(b->stream, [&]() { return enqueue_all(b, b->stream); }, 3); };
        double best = time_batch();
        std::map<int, std::vector<int>> corr_cls;  // n_spec -> sub-bands
        std::map<std::pair<int, int>, std::vector<int>> grid_cls;  // (n_pix, n_chan) -> sub-bands
        for (int s = 0; s < n_sb; s++) {
            if (!cache.count(corr_key(n_in, b->sb[s].n_spec))) corr_cls[b->sb[s].n_spec].push_back(s);
            if (!(flags & NBSI_BATCH_GRID_TALL) && !cache.count(grid_key(n_ant, b->sb[s].n_pix, b->sb[s].n_chan)))
                grid_cls[{b->sb[s].n_pix, b->sb[s].n_chan}].push_back(s);
        }
        for (auto &kv : corr_cls) {
            const int cur = b->corr_variant[kv.second[0]];
            int keep = cur;
            for (int v : {CORR_VARIANT_TILED, CORR_VARIANT_CHAN32, CORR_VARIANT_CHAN64}) {
                if (v == cur || !correlate_variant_valid(n_in, kv.first, v)) continue;
                for (int s : kv.second) b->corr_variant[s] = v;
                if ((rc = relaunch())) return fail(rc, "launch tables failed");
                const double t = time_batch();
                if (t < 0.99 * best) {
                    best = t;
                    keep = v;
                }
            }
            for (int s : kv.second) b->corr_variant[s] = keep;
            cache[corr_key(n_in, kv.first)] = keep;
            cache_dirty = true;
        }
        for (auto &kv : grid_cls) {
            const int cur = b->grid_ge[kv.second[0]], alt = cur == 16 ? 32 : 16;
            std::vector<nbsi_image_plan *> old;
            for (int s : kv.second) {
                nbsi_image_plan *p = nullptr;
                if ((rc = build_plan(s, alt, &p))) {
                    for (size_t q = 0; q < old.size(); q++) std::swap(b->plans[kv.second[q]], old[q]);
                    for (auto *o : old) nbsi_image_plan_destroy(o);
                    return fail(rc, "plan failed");
                }
                old.push_back(b->plans[s]);
                b->plans[s] = p;
                b->grid_ge[s] = alt;
            }
            if ((rc = relaunch())) return fail(rc, "launch tables failed");
            const double t = time_batch();
            int keep = alt;
            if (t < 0.99 * best) {
                best = t;
            } else {  // revert to the previous plans
                keep = cur;
                for (size_t q = 0; q < old.size(); q++) {
                    std::swap(b->plans[kv.second[q]], old[q]);
                    b->grid_ge[kv.second[q]] = cur;
                }
            }
            for (auto *o : old) nbsi_image_plan_destroy(o);
            cache[grid_key(n_ant, kv.first.first, kv.first.second)] = keep;
            cache_dirty = true;
        }
        if ((rc = relaunch())) return fail(rc, "launch tables failed");
    }
    if (cache_dirty) write_cache(tune_cache_path, cache);
    if (hipStreamSynchronize(b->stream) != hipSuccess) return fail(NBSI_EHIP, "stream sync failed");
    // description of the choices (JSON)
    std::string d = "{\"subbands\": [";
    for (int s = 0; s < n_sb; s++) {
        char tmp[256];
        snprintf(tmp, sizeof tmp, "%s{\"n_fft\": %d, \"n_spec\": %d, \"n_chan\": %d, \"n_pix\": %d, \"corr_variant\": \"%s\", \"grid_ge\": %d}",
                 s ? ", " : "", b->sb[s].n_fft, b->sb[s].n_spec, b->sb[s].n_chan, b->sb[s].n_pix,
                 b->corr_variant[s] == CORR_VARIANT_TILED ? "tiled" : (b->corr_variant[s] == CORR_VARIANT_CHAN32 ? "channel32" : "channel64"),
                 b->grid_ge[s]);
        d += tmp;
    }
    d += "], \"launches\": " + std::to_string(b->launches.size()) + "}";
    b->desc = d;
    if (prev >= 0 && prev != ctx->device) (void)hipSetDevice(prev);
    *out = b;
    return NBSI_OK;
}

int nbsi_batch_run(nbsi_batch *b) {
    if (!b) return NBSI_EINVAL;
    nbsi_ctx *ctx = b->ctx;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != b->device) (void)hipSetDevice(b->device);
    auto done = [&](int code) {
        if (prev >= 0 && prev != b->device) (void)hipSetDevice(prev);
        return code;
    };
    // order after the caller's stream, run on the batch stream, then order the caller after it
    if (hipEventRecord(b->ev_in, ctx->stream) != hipSuccess || hipStreamWaitEvent(b->stream, b->ev_in, 0) != hipSuccess)
        return done(nbsi_fail(ctx, NBSI_EHIP, "nbsi_batch_run: event ordering failed"));
    // with NBSI_BATCH_OVERLAP the launches go straight to the two streams: a captured graph of
    // the two branches, replayed, overlapped them less (66.1 against 64.1 ms on twelve sub-bands)
    if ((b->flags & NBSI_BATCH_GRAPH) && !b->aux) {
        if (!b->captured) {
            if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return done(nbsi_fail(ctx, NBSI_EHIP, "nbsi_batch_run: capture failed to start"));
            const hipError_t e = enqueue_all(b, b->stream);
            hipGraph_t g = nullptr;
            const hipError_t e2 = hipStreamEndCapture(b->stream, &g);
            if (e != hipSuccess || e2 != hipSuccess || !g)
                return done(nbsi_fail(ctx, NBSI_EHIP, "nbsi_batch_run: capture failed"));
            b->graph = g;
            if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
                return done(nbsi_fail(ctx, NBSI_EHIP, "nbsi_batch_run: graph instantiation failed"));
            b->captured = true;
        }
        if (hipGraphLaunch(b->exec, b->stream) != hipSuccess)
            return done(nbsi_fail(ctx, NBSI_EHIP, "nbsi_batch_run: graph launch failed"));
    } else {
        if (enqueue_all(b, b->stream) != hipSuccess) return done(nbsi_fail(ctx, NBSI_EHIP, "nbsi_batch_run: launch failed"));
    }
    if (hipEventRecord(b->ev_out, b->stream) != hipSuccess || hipStreamWaitEvent(ctx->stream, b->ev_out, 0) != hipSuccess)
        return done(nbsi_fail(ctx, NBSI_EHIP, "nbsi_batch_run: event ordering failed"));
    return done(NBSI_OK);
}

int nbsi_batch_describe(const nbsi_batch *b, char *buf, int len) {
    if (!b || !buf || len <= 0) return NBSI_EINVAL;
    const int n = (int)b->desc.size();
    if (n + 1 > len) {
        memcpy(buf, b->desc.data(), len - 1);
        buf[len - 1] = 0;
        return NBSI_ETRUNC;
    }
    memcpy(buf, b->desc.c_str(), n + 1);
    return NBSI_OK;
}

int nbsi_batch_destroy(nbsi_batch *b) {
    if (!b) return NBSI_EINVAL;
    int prev = -1;
    (void)hipGetDevice(&prev);
    const int dev = b->device;
    if (prev != dev) (void)hipSetDevice(dev);
    free_batch(b);
    if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
    return NBSI_OK;
}

}  // extern "C"
