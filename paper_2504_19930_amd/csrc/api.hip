// C ABI of the registration library (declared in include/smc.h): argument
// checks, ownership of device workspaces, and the launch sequence of the
// particle filter of Fig. 1.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <limits.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "smc.h"

using namespace smc;

namespace {

thread_local std::string g_err;

// Launch defaults (see smc_set_tuning).
// (measured on MI355X: packed octets, 4 particles per workgroup; see smc_autotune)
constexpr int kDefaultLayout = kLayoutLerp;
constexpr int kDefaultPT = 4;
// default tile depths, from measurements on MI355X: masks 16 (culling against
// the source mask's bounding box pays at shallow tiles), images 256
constexpr int kDefaultZChunkMask = 16, kDefaultZChunkImage = 256;

smc_status fail(smc_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return fail(SMC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

bool finite6(const double *v) {
    for (int d = 0; d < 6; ++d)
        if (!isfinite(v[d])) return false;
    return true;
}

smc_status check_volume(const smc_volume *v, const char *name) {
    if (!v) return fail(SMC_EINVAL, "%s is NULL", name);
    if (!v->data) return fail(SMC_EINVAL, "%s->data is NULL", name);
    if (v->nx < 1 || v->ny < 1 || v->nz < 1 || v->nx > 65535 || v->ny > 65535 || v->nz > 65535)
        return fail(SMC_EINVAL, "%s dimensions %d x %d x %d outside 1..65535", name, v->nx, v->ny, v->nz);
    if ((int64_t)v->nx * v->ny * v->nz >= ((int64_t)1 << 31))
        return fail(SMC_EINVAL, "%s has 2^31 voxels or more", name);
    if ((int64_t)v->nx * v->ny >= ((int64_t)1 << 24))
        return fail(SMC_EINVAL, "%s has 2^24 voxels or more per slice", name);
    if (!(v->sx > 0 && v->sy > 0 && v->sz > 0) || !isfinite(v->sx) || !isfinite(v->sy) || !isfinite(v->sz))
        return fail(SMC_EINVAL, "%s spacing must be finite and positive", name);
    return SMC_OK;
}

smc_status check_params(const smc_params *p) {
    if (!p) return fail(SMC_EINVAL, "params is NULL");
    // the resampling CDF sums floor(w 2^48) <= 2^48 per particle in 64 bits
    if (p->n_particles < 1 || p->n_particles > 65535) return fail(SMC_EINVAL, "n_particles must be in 1..65535");
    if (p->n_iters < 1 || p->n_iters > 100000) return fail(SMC_EINVAL, "n_iters must be in 1..100000");
    if (p->score < SMC_SCORE_DICE || p->score > SMC_SCORE_MI) return fail(SMC_EINVAL, "unknown score %d", p->score);
    if (p->interp != SMC_INTERP_NEAREST && p->interp != SMC_INTERP_TRILINEAR)
        return fail(SMC_EINVAL, "unknown interpolation %d", p->interp);
    if (p->rotation_mode != SMC_ROTATION_BOX && p->rotation_mode != SMC_ROTATION_WIDE)
        return fail(SMC_EINVAL, "unknown rotation_mode %d", p->rotation_mode);
    if (p->score == SMC_SCORE_MI && p->interp != SMC_INTERP_TRILINEAR)
        return fail(SMC_EINVAL, "the mutual-information score samples trilinearly");
    if (p->score == SMC_SCORE_DICE && p->interp != SMC_INTERP_NEAREST)
        return fail(SMC_EINVAL, "the Dice score works on binary masks with nearest-neighbour sampling");
    if (!finite6(p->x0) || !finite6(p->limit) || !finite6(p->sigma0))
        return fail(SMC_EINVAL, "x0, limit and sigma0 must be finite");
    for (int d = 0; d < 6; ++d) {
        if (!(p->limit[d] > 0.0)) return fail(SMC_EINVAL, "limit[%d] must be positive", d);
        if (p->sigma0[d] < 0.0) return fail(SMC_EINVAL, "sigma0[%d] must be non-negative", d);
        if (fabs(p->x0[d]) + p->limit[d] > 1e6) return fail(SMC_EINVAL, "prior box too large on axis %d", d);
    }
    if (!(p->sigma_score > 0.0) || !isfinite(p->sigma_score)) return fail(SMC_EINVAL, "sigma_score must be positive");
    if (!(p->anneal > 0.0 && p->anneal <= 1.0)) return fail(SMC_EINVAL, "anneal must be in (0, 1]");
    if (!(p->min_overlap_frac >= 0.0 && p->min_overlap_frac <= 1.0))
        return fail(SMC_EINVAL, "min_overlap_frac must be in [0, 1]");
    return SMC_OK;
}

struct Stats {
    uint64_t count, on;
    double mu, sd;
};

// Mean and population standard deviation over the FOV from exact sums.
Stats stats_from_sums(const unsigned long long s[4]) {
    Stats r;
    r.count = s[0];
    r.on = s[1];
    const double dn = (double)s[0];
    const double m = (double)s[2] / dn;
    const double var = (double)s[3] / dn - m * m;
    r.mu = m;
    r.sd = var > 0.0 ? sqrt(var) : 1.0;
    return r;
}

// Allocation-free evaluation (smc_evaluate_noalloc): the recipe words of up
// to SMC_NOALLOC_MAX_PARTICLES particles live in this file-scope device array
// (one copy per device, for the life of the process).  Host code never uses
// the array's name as an address: smc_init resolves, once per device and with
// that device current, the device address of that device's copy, and the
// entry point passes only that address to the kernels.
static __device__ __align__(256) float scratch[12ull * SMC_NOALLOC_MAX_PARTICLES];

std::mutex g_scratch_mu;
std::map<int, float *> g_scratch_ptr;  // device ordinal -> address of its `scratch`

// Resolve the current device's scratch address (no-op once resolved).
smc_status resolve_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr.count(device)) return SMC_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
        (void)hipGetLastError();
        return fail(SMC_EDEVICE, "hipGetSymbolAddress of the evaluation scratch array failed on device %d: %s",
                    device, hipGetErrorString(e));
    }
    g_scratch_ptr[device] = (float *)ptr;
    return SMC_OK;
}

float *scratch_of(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    return it == g_scratch_ptr.end() ? nullptr : it->second;
}

}  // namespace

struct smc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    smc_params p{};
    int mode = kModeMask;
    int32_t sn[3] = {0, 0, 0}, tn[3] = {0, 0, 0};
    const uint8_t *src = nullptr, *src_fov = nullptr, *tgt = nullptr, *tgt_fov = nullptr;
    uint8_t *src_prep = nullptr, *tgt_prep = nullptr, *src_ok = nullptr;
    uint32_t *src_bits = nullptr;  // masks: bitmap of the source's on bits
    int layout = kDefaultLayout, pt = kDefaultPT, zchunk = kDefaultZChunkMask;
    int32_t box_lo[3] = {1, 1, 1}, box_hi[3] = {-1, -1, -1};  // source mask bounding box (empty)
    uint32_t *occ = nullptr;  // masks: summed-area table of the source's occupied cells (or none)
    unsigned long long *work = nullptr;  // masks: pairs evaluated and covered by the culled launches
    void *packed[kLayouts] = {};
    uint64_t sentinel[kLayouts] = {};  // per packed layout: value marking elements outside the source FOV
    bool has_sentinel[kLayouts] = {};
    FilterState f{};
    uint32_t k_done = 0;
    // the current particles are a draw from the uniform prior box (spread over
    // the whole limits): their first evaluation gathers from the tiled octets
    // when the lerp layout is configured (smaller elements, fewer lines per
    // gather: they suit the dispersed cloud, whose footprint streams from
    // beyond the L2s)
    bool prior_dispersed = false;
    // target |T| and FOV voxel count of this pair (the score constants pool them over frames)
    uint64_t tgt_on = 0, tgt_count = 0;
    // multi-frame score: further frame pairs, each prepared by a context of its
    // own; their score launches write into this context's words and sums
    std::vector<smc_ctx *> frames;
    bool in_batch = false;
    smc_status sticky = SMC_OK;
    std::string sticky_msg;
    // smc_gather_probe checksum word
    uint32_t *probe_out = nullptr;
    // masks: culled item lists of the filter's launches (capacity item_cap),
    // sized for launches of items_np particles (a frame pair's context scores
    // the particles of the context it belongs to)
    uint32_t items_np = 0;
    void *items = nullptr;
    uint32_t *item_counters = nullptr;
    uint64_t item_cap = 0;
    // smc_evaluate workspace
    uint32_t eval_cap = 0;
    double *x_eval = nullptr;
    float *w_eval = nullptr;
    unsigned long long *s_eval = nullptr;
    double *z_eval = nullptr;
    // mutual information: joint histograms of the filter's particles (N + 1)
    // and of the evaluation workspace (eval_cap), zero between evaluations
    uint32_t *hist = nullptr, *hist_eval = nullptr;
    std::vector<void *> allocs;
    // kernel timing
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_score, ev_filter;

    template <typename T>
    smc_status alloc(T **out, size_t count) {
        void *ptr = nullptr;
        const size_t bytes = count * sizeof(T) > 0 ? count * sizeof(T) : 1;
        if (hipMalloc(&ptr, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SMC_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
        }
        allocs.push_back(ptr);
        *out = static_cast<T *>(ptr);
        return SMC_OK;
    }

    // layout of a launch over a dispersed cloud (see prior_dispersed)
    int dispersed_layout() const {
        return mode == kModeImageTrilinear && layout == kLayoutLerp && packed[kLayoutOctTile] ? kLayoutOctTile
                                                                                               : layout;
    }

    // filter == true: only the sums the filter uses must be exact (masks: a, c);
    // dispersed == true: the particles are spread over the prior box
    ScoreLaunch score_launch(const float *words, unsigned long long *sums, uint32_t p0, uint32_t np,
                             bool filter = false, bool dispersed = false) const {
        const int layout = dispersed ? dispersed_layout() : this->layout;
        ScoreLaunch L;
        L.mode = mode;
        L.zchunk = zchunk;
        L.cull_box = filter && mode == kModeMask;
        for (int d = 0; d < 3; ++d) {
            L.box_lo[d] = box_lo[d];
            L.box_hi[d] = box_hi[d];
        }
        if (mode == kModeMask) {
            L.src = src_prep;
            L.src_bits = src_bits;
            L.occ = L.cull_box ? occ : nullptr;
            L.work = L.cull_box ? work : nullptr;
            L.src_ok = nullptr;
            L.tgt = tgt_prep;
            L.tgt_fov = nullptr;
        } else {
            L.src = src;
            L.src_ok = src_ok;
            L.tgt = tgt;
            L.tgt_fov = tgt_fov;
        }
        L.layout = mode == kModeImageTrilinear ? layout : kLayoutRaw;
        L.src_packed = mode == kModeImageTrilinear ? packed[L.layout] : nullptr;
        L.has_sentinel = mode == kModeImageTrilinear && has_sentinel[L.layout];
        L.sentinel = sentinel[L.layout];
        L.pt = pt;
        L.words = words;
        L.sums = sums;
        for (int d = 0; d < 3; ++d) {
            L.sn[d] = sn[d];
            L.tn[d] = tn[d];
        }
        L.p0 = p0;
        L.np = np;
        L.items = items;
        L.item_counters = item_counters;
        L.item_cap = item_cap;
        return L;
    }

    smc_status mark(smc_status st) {
        if (st != SMC_OK && sticky == SMC_OK) {
            sticky = st;
            sticky_msg = g_err;
        }
        return st;
    }
    smc_status check_sticky() {
        if (sticky != SMC_OK) return fail(sticky, "context failed earlier: %s", sticky_msg.c_str());
        return SMC_OK;
    }
};

namespace {

const int32_t kZeroFlag = 0;

smc_status set_device(smc_ctx *c) {
    HIP_TRY(hipSetDevice(c->device));
    return SMC_OK;
}

hipEvent_t take_event(smc_ctx *c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch `fn` on the context stream, bracketed by events when profiling.
template <typename F>
hipError_t timed(smc_ctx *c, std::vector<std::pair<hipEvent_t, hipEvent_t>> &log, F fn) {
    if (!c->profiling) return fn();
    hipEvent_t a = take_event(c), b = take_event(c);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, c->stream);
    if (e == hipSuccess) e = fn();
    if (e == hipSuccess) e = hipEventRecord(b, c->stream);
    log.emplace_back(a, b);
    return e;
}

uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// Allocate and fill a packed trilinear layout of the source.  With a source
// FOV, find a value no in-FOV element takes and store it in every element
// that touches a voxel outside the FOV (then samples need no separate
// validity gather); if none is free, pack plainly and keep the gather.
smc_status prepare_layout(smc_ctx *c, int layout) {
    if (c->mode != kModeImageTrilinear || layout == kLayoutRaw || c->packed[layout]) return SMC_OK;
    if (layout == kLayoutLerp && layout_fits(kLayoutOctTile, c->sn)) {
        // the tiled octets serve the first evaluation of a dispersed prior
        const smc_status so = prepare_layout(c, kLayoutOctTile);
        if (so != SMC_OK) return so;
    }
    smc_status st;
    if ((st = c->alloc((uint8_t **)&c->packed[layout], packed_bytes(layout, c->sn))) != SMC_OK) return st;
    uint64_t sent = 0;
    bool ok = false;
    if (c->src_fov && layout == kLayoutLerp) {
        sent = kLerpSentinel;
        ok = true;
    } else if (c->src_fov) {
        const int n_cand = layout == kLayoutPairX ? 0 : 64;
        const size_t n_counts = layout == kLayoutPairX ? 65536 : 64;
        std::vector<uint64_t> cand(64);
        for (int q = 0; q < 64; ++q) cand[q] = splitmix64((uint64_t)q + 1);
        uint64_t *dcand = nullptr;
        unsigned long long *dcounts = nullptr;
        std::vector<unsigned long long> counts(n_counts);
        hipError_t e = hipMalloc(&dcand, 8 * 64);
        if (e == hipSuccess) e = hipMalloc(&dcounts, 8 * n_counts);
        if (e == hipSuccess) e = hipMemcpyAsync(dcand, cand.data(), 8 * 64, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = launch_fill_u64(dcounts, n_counts, c->stream);
        if (e == hipSuccess)
            e = launch_count_elements(c->src, c->src_fov, c->sn, layout, dcand, n_cand, dcounts, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(counts.data(), dcounts, 8 * n_counts, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (dcand) (void)hipFree(dcand);
        if (dcounts) (void)hipFree(dcounts);
        if (e != hipSuccess) return fail(SMC_EDEVICE, "sentinel search failed: %s", hipGetErrorString(e));
        for (size_t q = 0; q < n_counts && !ok; ++q)
            if (counts[q] == 0) {
                sent = layout == kLayoutPairX ? (uint64_t)q : cand[q];
                ok = true;
            }
    }
    HIP_TRY(launch_pack_source(c->src, ok ? c->src_fov : nullptr, c->sn, layout, sent, c->packed[layout],
                               c->stream));
    c->sentinel[layout] = sent;
    c->has_sentinel[layout] = ok;
    return SMC_OK;
}

smc_status launch_prior(smc_ctx *c) {
    HIP_TRY(launch_fill_u64(c->f.sums, 6ull * (c->f.n + 1), c->stream));
    HIP_TRY(launch_init_particles(c->f, c->stream));
    c->k_done = 0;
    c->prior_dispersed = !c->f.has_proposal;
    return SMC_OK;
}

// Mask contexts: item lists large enough for a filter launch (N + 1
// particles) under the current tuning; smaller buffers are freed.
// Every filter launch must fit one grid (masks and images alike).
smc_status check_items(const smc_ctx *c) {
    const uint64_t items = score_items_for(c->score_launch(c->f.words, c->f.sums, 0, c->f.n + 1, true));
    if (items > kMaxScoreItems)
        return fail(SMC_EINVAL, "%llu work items per scoring launch exceed %llu: use deeper tiles or fewer particles",
                    (unsigned long long)items, (unsigned long long)kMaxScoreItems);
    return SMC_OK;
}

smc_status ensure_items(smc_ctx *c) {
    smc_status st;
    if ((st = check_items(c)) != SMC_OK) return st;
    if (c->mode != kModeMask) return SMC_OK;
    if (!c->item_counters && (st = c->alloc(&c->item_counters, kItemCounterWords)) != SMC_OK) return st;
    const uint32_t np = std::max(c->f.n + 1, c->items_np);
    const uint64_t need = score_items_for(c->score_launch(c->f.words, c->f.sums, 0, np, true));
    if (need > kMaxScoreItems) return SMC_OK;  // such launches run as a grid (and are refused there)
    if (need <= c->item_cap) return SMC_OK;
    if (c->items) {
        if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(SMC_EDEVICE, "stream sync failed");
        c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), c->items), c->allocs.end());
        (void)hipFree(c->items);
        c->items = nullptr;
        c->item_cap = 0;
    }
    uint2 *buf = nullptr;
    if ((st = c->alloc(&buf, need)) != SMC_OK) return st;
    c->items = buf;
    c->item_cap = need;
    return SMC_OK;
}

smc_status ensure_eval(smc_ctx *c, uint32_t n) {
    if (n <= c->eval_cap) return SMC_OK;
    // grow: old buffers stay in c->allocs until destroy (small)
    smc_status st;
    if ((st = c->alloc(&c->x_eval, 6ull * n)) != SMC_OK) return st;
    if ((st = c->alloc(&c->w_eval, 12ull * n)) != SMC_OK) return st;
    if ((st = c->alloc(&c->s_eval, 6ull * n)) != SMC_OK) return st;
    if ((st = c->alloc(&c->z_eval, n)) != SMC_OK) return st;
    if (c->p.score == SMC_SCORE_MI) {
        const uint64_t words = (uint64_t)kMiBins * kMiBins * n;
        if ((st = c->alloc(&c->hist_eval, words)) != SMC_OK) return st;
        HIP_TRY(launch_fill_u64((unsigned long long *)c->hist_eval, words / 2, c->stream));
    }
    c->eval_cap = n;
    return SMC_OK;
}

// Score particles p0 .. p0 + np - 1 of `words` into `sums`: the context's own
// frame pair, then every further frame pair of a multi-frame score (integer
// sums, so the pooled result does not depend on the order).
hipError_t launch_score_frames(smc_ctx *c, const float *words, unsigned long long *sums, uint32_t *hist,
                               uint32_t p0, uint32_t np, bool filter, bool dispersed = false) {
    const bool mi = c->p.score == SMC_SCORE_MI;
    ScoreLaunch L = c->score_launch(words, sums, p0, np, filter, dispersed);
    if (mi) L.hist = hist;
    hipError_t e = launch_score(L, c->stream);
    for (size_t q = 0; q < c->frames.size() && e == hipSuccess; ++q) {
        ScoreLaunch F = c->frames[q]->score_launch(words, sums, p0, np, filter, dispersed);
        if (mi) F.hist = hist;
        e = launch_score(F, c->stream);
    }
    // mutual information: the pooled histograms become scores
    if (mi && e == hipSuccess) e = launch_mi_finalize(hist, p0, np, sums, c->stream);
    return e;
}

// Score constants of the pooled frames: |T| and the minimum overlap count
// over all target frames.
void pool_frame_constants(smc_ctx *c) {
    uint64_t on = c->tgt_on, count = c->tgt_count;
    for (smc_ctx *fr : c->frames) {
        on += fr->tgt_on;
        count += fr->tgt_count;
    }
    c->f.sc.t_on = on;
    c->f.sc.min_n = (uint64_t)ceil(c->p.min_overlap_frac * (double)count);
}

// Score a device particle set with the context's kernel; sums into s_eval.
smc_status evaluate_device(smc_ctx *c, const double *x_dev, uint32_t n) {
    smc_status st = ensure_eval(c, n);
    if (st != SMC_OK) return st;
    HIP_TRY(launch_words(x_dev, n, c->f.geom, c->f.nearest, c->w_eval, c->stream));
    HIP_TRY(launch_fill_u64(c->s_eval, 6ull * n, c->stream));
    HIP_TRY(launch_score_frames(c, c->w_eval, c->s_eval, c->hist_eval, 0, n, false));
    return SMC_OK;
}

}  // namespace

extern "C" {

const char *smc_last_error(void) { return g_err.c_str(); }

const char *smc_version(void) { return "smcreg 0.1 (gfx950)"; }

smc_status smc_init(smc_ctx **out, const smc_volume *src, const smc_volume *tgt, const smc_params *p,
                    void *hip_stream) {
    g_err.clear();
    if (!out) return fail(SMC_EINVAL, "out is NULL");
    *out = nullptr;
    smc_status st;
    if ((st = check_volume(src, "src")) != SMC_OK) return st;
    if ((st = check_volume(tgt, "tgt")) != SMC_OK) return st;
    if ((st = check_params(p)) != SMC_OK) return st;

    smc_ctx *c = new (std::nothrow) smc_ctx();
    if (!c) return fail(SMC_ENOMEM, "host allocation failed");
    c->stream = (hipStream_t)hip_stream;
    c->p = *p;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(SMC_EDEVICE, "no HIP device");
    }
    if ((st = resolve_scratch(c->device)) != SMC_OK) {
        delete c;
        return st;
    }
    c->sn[0] = src->nx; c->sn[1] = src->ny; c->sn[2] = src->nz;
    c->tn[0] = tgt->nx; c->tn[1] = tgt->ny; c->tn[2] = tgt->nz;
    c->src = src->data;
    c->src_fov = src->fov;
    c->tgt = tgt->data;
    c->tgt_fov = tgt->fov;
    c->mode = p->score == SMC_SCORE_DICE ? kModeMask
              : (p->interp == SMC_INTERP_TRILINEAR ? kModeImageTrilinear : kModeImageNearest);
    c->zchunk = c->mode == kModeMask ? kDefaultZChunkMask : kDefaultZChunkImage;
    const int64_t vs = (int64_t)src->nx * src->ny * src->nz;
    const int64_t vt = (int64_t)tgt->nx * tgt->ny * tgt->nz;
    const uint32_t n = p->n_particles, K = p->n_iters;

    auto bail = [&](smc_status s) {
        smc_destroy(c);
        return s;
    };

    // prepared inputs
    if (c->mode == kModeMask) {
        if ((st = c->alloc(&c->src_prep, vs)) != SMC_OK) return bail(st);
        if ((st = c->alloc(&c->tgt_prep, vt)) != SMC_OK) return bail(st);
        if ((st = c->alloc((uint8_t **)&c->src_bits, mask_bits_bytes(c->sn))) != SMC_OK) return bail(st);
        if (launch_prep_mask(src->data, src->fov, c->src_prep, vs, c->stream) != hipSuccess ||
            launch_prep_mask(tgt->data, tgt->fov, c->tgt_prep, vt, c->stream) != hipSuccess ||
            launch_pack_mask_bits(c->src_prep, c->sn, c->src_bits, c->stream) != hipSuccess)
            return bail(fail(SMC_EDEVICE, "mask preparation launch failed"));
    } else if (src->fov) {
        if (c->mode == kModeImageTrilinear) {
            if ((st = c->alloc(&c->src_ok, vs)) != SMC_OK) return bail(st);
            if (launch_corner_valid(src->fov, c->src_ok, c->sn, c->stream) != hipSuccess)
                return bail(fail(SMC_EDEVICE, "corner-validity launch failed"));
        } else {
            c->src_ok = const_cast<uint8_t *>(src->fov);
        }
    }

    if (!layout_fits(c->layout, c->sn)) c->layout = layout_fits(kLayoutOct, c->sn) ? kLayoutOct : kLayoutRaw;
    if ((st = prepare_layout(c, c->layout)) != SMC_OK) return bail(st);

    if (c->mode == kModeMask) {
        int32_t *dbox = nullptr;
        const int32_t init[6] = {INT32_MAX, INT32_MAX, INT32_MAX, -1, -1, -1};
        int32_t hb[6];
        if ((st = c->alloc(&dbox, 6)) != SMC_OK) return bail(st);
        if (hipMemcpyAsync(dbox, init, sizeof init, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
            launch_mask_bbox(c->src_prep, c->sn, dbox, c->stream) != hipSuccess ||
            hipMemcpyAsync(hb, dbox, sizeof hb, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            return bail(fail(SMC_EDEVICE, "source mask bounding box failed"));
        if (hb[3] >= 0)
            for (int d = 0; d < 3; ++d) {
                c->box_lo[d] = hb[d];
                c->box_hi[d] = hb[3 + d];
            }
        // occupancy of 2^3-voxel cells for the culled launches, when its table
        // is modest (flat volumes would make its zero borders large)
        if ((st = c->alloc(&c->work, kWorkSlots * kWorkSlotWords)) != SMC_OK) return bail(st);
        if (launch_fill_u64(c->work, kWorkSlots * kWorkSlotWords, c->stream) != hipSuccess)
            return bail(fail(SMC_EDEVICE, "work counter fill failed"));
        const uint64_t ow = mask_occ_words(c->sn);
        if (ow <= kOccMaxWords) {
            if ((st = c->alloc(&c->occ, ow)) != SMC_OK) return bail(st);
            if (launch_mask_occupancy(c->src_prep, c->sn, c->occ, c->stream) != hipSuccess)
                return bail(fail(SMC_EDEVICE, "source mask occupancy launch failed"));
        }
    }

    // exact per-volume sums -> statistics
    unsigned long long *vsum = nullptr;
    if ((st = c->alloc(&vsum, 8)) != SMC_OK) return bail(st);
    unsigned long long hs[8];
    if (launch_fill_u64(vsum, 8, c->stream) != hipSuccess ||
        launch_volume_sums(tgt->data, tgt->fov, vt, vsum, c->stream) != hipSuccess ||
        launch_volume_sums(src->data, src->fov, vs, vsum + 4, c->stream) != hipSuccess)
        return bail(fail(SMC_EDEVICE, "volume statistics launch failed"));
    if (hipMemcpyAsync(hs, vsum, sizeof hs, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return bail(fail(SMC_EDEVICE, "reading volume statistics failed: %s", hipGetErrorString(hipGetLastError())));
    const Stats ts = stats_from_sums(hs), ss = stats_from_sums(hs + 4);
    if (ts.count == 0) return bail(fail(SMC_EINVAL, "the target FOV is empty"));
    c->tgt_on = ts.on;
    c->tgt_count = ts.count;

    FilterState &f = c->f;
    f.n = n;
    f.n_iters = K;
    f.seed = p->seed;
    f.pair = p->pair_id;
    for (int d = 0; d < 3; ++d) f.geom.tn[d] = c->tn[d];
    f.geom.ts[0] = tgt->sx; f.geom.ts[1] = tgt->sy; f.geom.ts[2] = tgt->sz;
    f.geom.ss[0] = src->sx; f.geom.ss[1] = src->sy; f.geom.ss[2] = src->sz;
    f.nearest = c->mode != kModeImageTrilinear;
    f.sc.kind = p->score;
    f.sc.t_on = ts.on;
    f.sc.min_n = (uint64_t)ceil(p->min_overlap_frac * (double)ts.count);
    f.sc.mu_s = ss.mu;
    f.sc.sd_s = ss.sd;
    f.sc.mu_t = ts.mu;
    f.sc.sd_t = ts.sd;
    f.sc.sigma = p->sigma_score;
    for (int d = 0; d < 6; ++d) {
        f.x0[d] = p->x0[d];
        f.limit[d] = p->limit[d];
        f.lo[d] = p->x0[d] - p->limit[d];
        f.hi[d] = p->x0[d] + p->limit[d];
        f.sigma0[d] = p->sigma0[d];
    }
    f.anneal = p->anneal;
    f.wide = p->rotation_mode == SMC_ROTATION_WIDE ? 1 : 0;
    if ((st = c->alloc(&f.x, 6ull * n)) != SMC_OK ||
        (st = c->alloc(&f.x_next, 6ull * n)) != SMC_OK ||
        (st = c->alloc(&f.words, 12ull * (n + 1))) != SMC_OK ||
        (st = c->alloc(&f.sums, 6ull * (n + 1))) != SMC_OK ||
        (st = c->alloc(&f.lw, n)) != SMC_OK || (st = c->alloc(&f.w, n)) != SMC_OK ||
        (st = c->alloc(&f.cdf, n)) != SMC_OK || (st = c->alloc(&f.anc, n)) != SMC_OK ||
        (st = c->alloc(&f.est, 6)) != SMC_OK || (st = c->alloc(&f.trace_score, K + 1ull)) != SMC_OK ||
        (st = c->alloc(&f.trace_ess, K)) != SMC_OK || (st = c->alloc(&f.trace_est, 6ull * K)) != SMC_OK ||
        (st = c->alloc(&f.flags, 4)) != SMC_OK)
        return bail(st);
    if (p->score == SMC_SCORE_MI) {
        const uint64_t words = (uint64_t)kMiBins * kMiBins * (n + 1ull);
        if ((st = c->alloc(&c->hist, words)) != SMC_OK) return bail(st);
        if (launch_fill_u64((unsigned long long *)c->hist, words / 2, c->stream) != hipSuccess)
            return bail(fail(SMC_EDEVICE, "histogram clear failed"));
    }
    if ((st = ensure_items(c)) != SMC_OK) return bail(st);
    if ((st = launch_prior(c)) != SMC_OK) return bail(st);
    *out = c;
    return SMC_OK;
}

smc_status smc_reset(smc_ctx *c, uint64_t seed) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    smc_status st;
    if ((st = c->check_sticky()) != SMC_OK) return st;
    if ((st = set_device(c)) != SMC_OK) return c->mark(st);
    c->f.seed = seed;
    c->p.seed = seed;
    return c->mark(launch_prior(c));
}

smc_status smc_step(smc_ctx *c, uint32_t n_iters) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    smc_status st;
    if ((st = c->check_sticky()) != SMC_OK) return st;
    if ((uint64_t)c->k_done + n_iters > c->f.n_iters)
        return fail(SMC_ESTATE, "%u iterations requested, %u of %u already run", n_iters, c->k_done, c->f.n_iters);
    if ((st = set_device(c)) != SMC_OK) return c->mark(st);
    for (uint32_t it = 0; it < n_iters; ++it) {
        const uint32_t k = c->k_done + 1;
        const bool dispersed = k == 1 && c->prior_dispersed;
        hipError_t e = timed(c, c->ev_score, [&] {
            return launch_score_frames(c, c->f.words, c->f.sums, c->hist, 0, c->f.n + 1, true, dispersed);
        });
        if (e == hipSuccess) e = timed(c, c->ev_filter, [&] { return launch_filter(c->f, k, c->stream); });
        if (e == hipSuccess && k == c->f.n_iters) {
            e = launch_score_frames(c, c->f.words, c->f.sums, c->hist, c->f.n, 1, true);
            if (e == hipSuccess) e = launch_ghost_final(c->f, c->stream);
        }
        if (e != hipSuccess) return c->mark(fail(SMC_EDEVICE, "iteration %u launch failed: %s", k, hipGetErrorString(e)));
        c->k_done = k;
    }
    return SMC_OK;
}

smc_status smc_evaluate(smc_ctx *c, const double *states, uint32_t n, int64_t *moments) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    if (c->p.score == SMC_SCORE_MI) return fail(SMC_EINVAL, "the MI score has no moments; use smc_score_particles");
    if (n == 0) return SMC_OK;
    if (!states || !moments) return fail(SMC_EINVAL, "states and moments must not be NULL");
    for (uint64_t q = 0; q < 6ull * n; ++q)
        if (!isfinite(states[q])) return fail(SMC_EINVAL, "state %llu is not finite", (unsigned long long)q);
    smc_status st;
    if ((st = c->check_sticky()) != SMC_OK) return st;
    if ((st = set_device(c)) != SMC_OK) return c->mark(st);
    if ((st = ensure_eval(c, n)) != SMC_OK) return c->mark(st);
    if (hipMemcpyAsync(c->x_eval, states, 48ull * n, hipMemcpyHostToDevice, c->stream) != hipSuccess)
        return c->mark(fail(SMC_EDEVICE, "upload of states failed"));
    if ((st = evaluate_device(c, c->x_eval, n)) != SMC_OK) return c->mark(st);
    if (hipMemcpyAsync(moments, c->s_eval, 48ull * n, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return c->mark(fail(SMC_EDEVICE, "evaluation failed: %s", hipGetErrorString(hipGetLastError())));
    return SMC_OK;
}

smc_status smc_evaluate_noalloc(smc_ctx *c, const double *states_dev, uint32_t n, int64_t *moments_dev) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    if (c->p.score == SMC_SCORE_MI) return fail(SMC_EINVAL, "the MI score has no moments");
    if (n > SMC_NOALLOC_MAX_PARTICLES)
        return fail(SMC_EINVAL, "n = %u exceeds the allocation-free maximum of %u particles", n,
                    (unsigned)SMC_NOALLOC_MAX_PARTICLES);
    if (n == 0) return SMC_OK;
    if (!states_dev || !moments_dev) return fail(SMC_EINVAL, "states_dev and moments_dev must not be NULL");
    smc_status st;
    if ((st = c->check_sticky()) != SMC_OK) return st;
    if ((st = set_device(c)) != SMC_OK) return c->mark(st);
    float *words = scratch_of(c->device);
    if (!words) return fail(SMC_EDEVICE, "no evaluation scratch resolved for device %d", c->device);
    unsigned long long *sums = reinterpret_cast<unsigned long long *>(moments_dev);
    // every word of particles 0 .. n-1 is rewritten; the sums start from zero
    HIP_TRY(launch_words(states_dev, n, c->f.geom, c->f.nearest, words, c->stream));
    HIP_TRY(launch_fill_u64(sums, 6ull * n, c->stream));
    HIP_TRY(launch_score_frames(c, words, sums, nullptr, 0, n, false));
    return SMC_OK;
}

smc_status smc_gather_probe(smc_ctx *c, uint32_t reps, double *probe_ms, double *score_ms) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    if (reps < 1 || reps > 1000) return fail(SMC_EINVAL, "reps must be in 1..1000");
    if (c->p.score == SMC_SCORE_MI || !c->frames.empty())
        return fail(SMC_EINVAL, "the gather probe covers single-pair moment and mask scores");
    smc_status st;
    if ((st = c->check_sticky()) != SMC_OK) return st;
    if ((st = set_device(c)) != SMC_OK) return c->mark(st);
    const uint32_t np = c->f.n + 1;  // the particles and the estimate, as the filter scores them
    const bool dispersed = c->k_done == 0 && c->prior_dispersed;
    if ((st = ensure_eval(c, np)) != SMC_OK) return c->mark(st);
    if (!c->probe_out && (st = c->alloc(&c->probe_out, 1)) != SMC_OK) return c->mark(st);
    ScoreLaunch L = c->score_launch(c->f.words, c->s_eval, 0, np, true, dispersed);
    if (!gather_probe_supported(L))
        return fail(SMC_EINVAL, "no gather probe for this score mode, layout or target FOV");
    hipEvent_t e0 = take_event(c), e1 = take_event(c);
    if (!e0 || !e1) {
        if (e0) c->ev_pool.push_back(e0);
        if (e1) c->ev_pool.push_back(e1);
        return fail(SMC_EDEVICE, "hipEventCreate failed");
    }
    // one untimed launch of each, then reps timed launches; the key is never
    // matched (a checksum equal to it would only write probe_out)
    double t_probe = 0.0, t_score = 0.0;
    auto time_one = [&](bool probe, double *acc) -> hipError_t {
        for (uint32_t r = 0; r <= reps; ++r) {
            hipError_t e = probe ? hipSuccess : launch_fill_u64(c->s_eval, 6ull * np, c->stream);
            if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
            if (e == hipSuccess)
                e = probe ? launch_gather_probe(L, 0xA5A5A5A5u, c->probe_out, c->stream) : launch_score(L, c->stream);
            if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) return e;
            if (r > 0) *acc += ms;
        }
        return hipSuccess;
    };
    hipError_t e = time_one(true, &t_probe);
    if (e == hipSuccess) e = time_one(false, &t_score);
    c->ev_pool.push_back(e0);  // the events go back to the pool on every path
    c->ev_pool.push_back(e1);
    if (e != hipSuccess) return fail(SMC_EDEVICE, "gather probe: %s", hipGetErrorString(e));
    if (probe_ms) *probe_ms = t_probe / reps;
    if (score_ms) *score_ms = t_score / reps;
    return SMC_OK;
}

smc_status smc_score_particles(smc_ctx *c, const double *states, uint32_t n, double *scores) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    if (n == 0) return SMC_OK;
    if (!states || !scores) return fail(SMC_EINVAL, "states and scores must not be NULL");
    for (uint64_t q = 0; q < 6ull * n; ++q)
        if (!isfinite(states[q])) return fail(SMC_EINVAL, "state %llu is not finite", (unsigned long long)q);
    smc_status st;
    if ((st = c->check_sticky()) != SMC_OK) return st;
    if ((st = set_device(c)) != SMC_OK) return c->mark(st);
    if ((st = ensure_eval(c, n)) != SMC_OK) return c->mark(st);
    if (hipMemcpyAsync(c->x_eval, states, 48ull * n, hipMemcpyHostToDevice, c->stream) != hipSuccess)
        return c->mark(fail(SMC_EDEVICE, "upload of states failed"));
    if ((st = evaluate_device(c, c->x_eval, n)) != SMC_OK) return c->mark(st);
    if (launch_scores_from_sums(c->s_eval, n, c->f.sc, c->z_eval, c->stream) != hipSuccess ||
        hipMemcpyAsync(scores, c->z_eval, 8ull * n, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return c->mark(fail(SMC_EDEVICE, "scoring failed: %s", hipGetErrorString(hipGetLastError())));
    return SMC_OK;
}

smc_status smc_exhaustive(smc_ctx *c, const double lo[6], const double step[6], const uint32_t count[6],
                          double best_params[6], double *best_score, double *scores) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    if (!lo || !step || !count) return fail(SMC_EINVAL, "lo, step and count must not be NULL");
    if (!finite6(lo) || !finite6(step)) return fail(SMC_EINVAL, "grid must be finite");
    uint64_t total = 1;
    for (int d = 0; d < 6; ++d) {
        if (count[d] < 1) return fail(SMC_EINVAL, "count[%d] must be >= 1", d);
        total *= count[d];
        if (total > ((uint64_t)1 << 40)) return fail(SMC_EINVAL, "grid too large");
    }
    smc_status st;
    if ((st = c->check_sticky()) != SMC_OK) return st;
    if ((st = set_device(c)) != SMC_OK) return c->mark(st);
    const uint32_t chunk = (uint32_t)std::min<uint64_t>(total, 8192);
    if ((st = ensure_eval(c, chunk)) != SMC_OK) return c->mark(st);
    const uint64_t n_chunks = (total + chunk - 1) / chunk;
    double *dz = nullptr, *dscores = nullptr;
    unsigned long long *di = nullptr;
    if ((st = c->alloc(&dz, n_chunks)) != SMC_OK || (st = c->alloc(&di, n_chunks)) != SMC_OK) return c->mark(st);
    if (scores && (st = c->alloc(&dscores, total)) != SMC_OK) return c->mark(st);
    for (uint64_t q = 0; q < n_chunks; ++q) {
        const uint64_t first = q * chunk;
        const uint32_t n = (uint32_t)std::min<uint64_t>(chunk, total - first);
        HIP_TRY(launch_grid_words(lo, step, count, first, n, c->f.geom, c->f.nearest, c->x_eval, c->w_eval,
                                  c->stream));
        HIP_TRY(launch_fill_u64(c->s_eval, 6ull * n, c->stream));
        HIP_TRY(launch_score_frames(c, c->w_eval, c->s_eval, c->hist_eval, 0, n, true));
        HIP_TRY(launch_chunk_best(c->s_eval, n, first, c->f.sc, dscores ? dscores + first : nullptr, dz + q, di + q,
                                  c->stream));
    }
    std::vector<double> hz(n_chunks);
    std::vector<unsigned long long> hi(n_chunks);
    HIP_TRY(hipMemcpyAsync(hz.data(), dz, 8 * n_chunks, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(hi.data(), di, 8 * n_chunks, hipMemcpyDeviceToHost, c->stream));
    if (scores) HIP_TRY(hipMemcpyAsync(scores, dscores, 8 * total, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    // the temporaries are released with the context (allocs list); drop them now
    for (void *ptr : {(void *)dz, (void *)di, (void *)dscores}) {
        if (!ptr) continue;
        c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), ptr), c->allocs.end());
        (void)hipFree(ptr);
    }
    double bz = -INFINITY;
    unsigned long long bi = ~0ull;
    for (uint64_t q = 0; q < n_chunks; ++q)
        if (hz[q] > bz || (hz[q] == bz && hi[q] < bi)) {
            bz = hz[q];
            bi = hi[q];
        }
    if (bi == ~0ull) bi = 0;
    if (best_params) {
        uint64_t g = bi;
        for (int d = 0; d < 6; ++d) {
            const uint64_t cd = g % count[d];
            g /= count[d];
            best_params[d] = lo[d] + step[d] * (double)cd;
        }
    }
    if (best_score) *best_score = bz;
    return SMC_OK;
}

smc_status smc_estimate(smc_ctx *c, double params[6], double mat3x4[12], double *score, double *ess) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    smc_status st;
    if ((st = c->check_sticky()) != SMC_OK) return st;
    if ((st = set_device(c)) != SMC_OK) return c->mark(st);
    double est[6], sc = NAN, e = NAN;
    int32_t flags[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(est, c->f.est, sizeof est, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(flags, c->f.flags, sizeof flags, hipMemcpyDeviceToHost, c->stream));
    if (c->k_done >= 1)
        HIP_TRY(hipMemcpyAsync(&e, c->f.trace_ess + (c->k_done - 1), sizeof e, hipMemcpyDeviceToHost, c->stream));
    if (c->k_done == c->f.n_iters)
        HIP_TRY(hipMemcpyAsync(&sc, c->f.trace_score + c->f.n_iters, sizeof sc, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (score && c->k_done < c->f.n_iters) {
        int64_t m[6];
        if ((st = smc_evaluate(c, est, 1, m)) != SMC_OK) return st;
        sc = score_from_sums(m, c->f.sc);
    }
    if (params) memcpy(params, est, sizeof est);
    if (mat3x4) rigid_matrix(est, c->f.geom, mat3x4);
    if (score) *score = sc;
    if (ess) *ess = e;
    if (c->k_done >= 1 && flags[1])
        return fail(SMC_ENOOVERLAP, "no particle reached the minimum overlap at iteration %u", c->k_done);
    return SMC_OK;
}

smc_status smc_get_particles(smc_ctx *c, double *states, double *logw, int32_t *anc) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    smc_status st;
    if ((st = c->check_sticky()) != SMC_OK) return st;
    if ((st = set_device(c)) != SMC_OK) return c->mark(st);
    const size_t n = c->f.n;
    if (states) HIP_TRY(hipMemcpyAsync(states, c->f.x, 48 * n, hipMemcpyDeviceToHost, c->stream));
    if (logw) HIP_TRY(hipMemcpyAsync(logw, c->f.lw, 8 * n, hipMemcpyDeviceToHost, c->stream));
    if (anc) HIP_TRY(hipMemcpyAsync(anc, c->f.anc, 4 * n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SMC_OK;
}

smc_status smc_trace(smc_ctx *c, double *score_k1, double *ess_k, double *est_6k) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    smc_status st;
    if ((st = c->check_sticky()) != SMC_OK) return st;
    if ((st = set_device(c)) != SMC_OK) return c->mark(st);
    const size_t K = c->f.n_iters;
    if (score_k1) HIP_TRY(hipMemcpyAsync(score_k1, c->f.trace_score, 8 * (K + 1), hipMemcpyDeviceToHost, c->stream));
    if (ess_k) HIP_TRY(hipMemcpyAsync(ess_k, c->f.trace_ess, 8 * K, hipMemcpyDeviceToHost, c->stream));
    if (est_6k) HIP_TRY(hipMemcpyAsync(est_6k, c->f.trace_est, 48 * K, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SMC_OK;
}

smc_status smc_set_particles(smc_ctx *c, const double *states, uint32_t k_done) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    if (!states) return fail(SMC_EINVAL, "states is NULL");
    if (k_done >= c->f.n_iters) return fail(SMC_EINVAL, "k_done must be below n_iters");
    for (uint64_t q = 0; q < 6ull * c->f.n; ++q)
        if (!isfinite(states[q])) return fail(SMC_EINVAL, "state %llu is not finite", (unsigned long long)q);
    smc_status st;
    if ((st = c->check_sticky()) != SMC_OK) return st;
    if ((st = set_device(c)) != SMC_OK) return c->mark(st);
    HIP_TRY(hipMemcpyAsync(c->f.x, states, 48ull * c->f.n, hipMemcpyHostToDevice, c->stream));
    // a caller's set is not a proposal draw: no importance correction
    HIP_TRY(hipMemcpyAsync(c->f.flags + 2, &kZeroFlag, sizeof kZeroFlag, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(launch_words(c->f.x, c->f.n, c->f.geom, c->f.nearest, c->f.words, c->stream));
    HIP_TRY(launch_fill_u64(c->f.sums, 6ull * (c->f.n + 1), c->stream));
    // the host copy must outlive the upload
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->k_done = k_done;
    c->prior_dispersed = false;  // a caller's particles: the configured layout throughout
    return SMC_OK;
}

namespace {
struct StateHeader {
    uint64_t magic, n, K, k_done;
};
const uint64_t kMagic = 0x534d435354415431ull;  // "SMCSTAT1"
}  // namespace

smc_status smc_get_state(smc_ctx *c, void *buf, size_t *len) {
    if (!c || !len) return fail(SMC_EINVAL, "ctx and len must not be NULL");
    const size_t n = c->f.n, K = c->f.n_iters;
    const size_t need = sizeof(StateHeader) + 48 * n + 8 * n + 4 * n + 48 + 8 * (K + 1) + 8 * K + 48 * K + 4;
    if (!buf) {
        *len = need;
        return SMC_OK;
    }
    if (*len < need) return fail(SMC_EINVAL, "buffer of %zu bytes, %zu needed", *len, need);
    smc_status st;
    if ((st = c->check_sticky()) != SMC_OK) return st;
    if ((st = set_device(c)) != SMC_OK) return c->mark(st);
    char *q = (char *)buf;
    StateHeader h{kMagic, n, K, c->k_done};
    memcpy(q, &h, sizeof h);
    q += sizeof h;
    struct Piece { const void *dev; size_t bytes; } pieces[] = {
        {c->f.x, 48 * n}, {c->f.lw, 8 * n}, {c->f.anc, 4 * n}, {c->f.est, 48},
        {c->f.trace_score, 8 * (K + 1)}, {c->f.trace_ess, 8 * K}, {c->f.trace_est, 48 * K}, {c->f.flags, 4}};
    for (auto &pc : pieces) {
        HIP_TRY(hipMemcpyAsync(q, pc.dev, pc.bytes, hipMemcpyDeviceToHost, c->stream));
        q += pc.bytes;
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    *len = need;
    return SMC_OK;
}

smc_status smc_set_state(smc_ctx *c, const void *buf, size_t len) {
    if (!c || !buf) return fail(SMC_EINVAL, "ctx and buf must not be NULL");
    const size_t n = c->f.n, K = c->f.n_iters;
    const size_t need = sizeof(StateHeader) + 48 * n + 8 * n + 4 * n + 48 + 8 * (K + 1) + 8 * K + 48 * K + 4;
    if (len < need) return fail(SMC_EINVAL, "state of %zu bytes, %zu expected", len, need);
    StateHeader h;
    memcpy(&h, buf, sizeof h);
    if (h.magic != kMagic || h.n != n || h.K != K || h.k_done > K)
        return fail(SMC_EINVAL, "state does not match this context");
    smc_status st;
    if ((st = c->check_sticky()) != SMC_OK) return st;
    if ((st = set_device(c)) != SMC_OK) return c->mark(st);
    const char *q = (const char *)buf + sizeof h;
    struct Piece { void *dev; size_t bytes; } pieces[] = {
        {c->f.x, 48 * n}, {c->f.lw, 8 * n}, {c->f.anc, 4 * n}, {c->f.est, 48},
        {c->f.trace_score, 8 * (K + 1)}, {c->f.trace_ess, 8 * K}, {c->f.trace_est, 48 * K}, {c->f.flags, 4}};
    for (auto &pc : pieces) {
        HIP_TRY(hipMemcpyAsync(pc.dev, q, pc.bytes, hipMemcpyHostToDevice, c->stream));
        q += pc.bytes;
    }
    // the state holds no proposal densities: a restored set gets no importance correction
    HIP_TRY(hipMemcpyAsync(c->f.flags + 2, &kZeroFlag, sizeof kZeroFlag, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(launch_words(c->f.x, c->f.n, c->f.geom, c->f.nearest, c->f.words, c->stream));
    HIP_TRY(launch_words(c->f.est, 1, c->f.geom, c->f.nearest, c->f.words + 12 * n, c->stream));
    HIP_TRY(launch_fill_u64(c->f.sums, 6ull * (n + 1), c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->k_done = (uint32_t)h.k_done;
    c->prior_dispersed = false;
    return SMC_OK;
}

smc_status smc_set_frames(smc_ctx *c, uint32_t n_extra, const smc_volume *src_frames,
                          const smc_volume *tgt_frames) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    if (n_extra > 4096) return fail(SMC_EINVAL, "n_extra must be at most 4096");
    if (n_extra > 0 && (!src_frames || !tgt_frames)) return fail(SMC_EINVAL, "src_frames and tgt_frames must not be NULL");
    if (c->in_batch) return fail(SMC_ESTATE, "frames cannot be added to a pair owned by a batch");
    if (c->k_done != 0) return fail(SMC_ESTATE, "frames must be set before the first iteration (smc_reset rewinds)");
    if (n_extra > 0 && c->p.score == SMC_SCORE_SSD)
        return fail(SMC_EINVAL, "the normalised SSD keeps per-volume statistics and is not pooled over frames");
    smc_status st;
    for (uint32_t q = 0; q < n_extra; ++q) {
        const smc_volume *s = &src_frames[q], *t = &tgt_frames[q];
        if ((st = check_volume(s, "src frame")) != SMC_OK || (st = check_volume(t, "tgt frame")) != SMC_OK) return st;
        if (s->nx != c->sn[0] || s->ny != c->sn[1] || s->nz != c->sn[2] || t->nx != c->tn[0] || t->ny != c->tn[1] ||
            t->nz != c->tn[2])
            return fail(SMC_EINVAL, "frame %u: shapes differ from the context's source / target", q + 1);
        if (s->sx != c->f.geom.ss[0] || s->sy != c->f.geom.ss[1] || s->sz != c->f.geom.ss[2] ||
            t->sx != c->f.geom.ts[0] || t->sy != c->f.geom.ts[1] || t->sz != c->f.geom.ts[2])
            return fail(SMC_EINVAL, "frame %u: spacings differ from the context's source / target", q + 1);
        if ((s->fov == nullptr) != (c->src_fov == nullptr) || (t->fov == nullptr) != (c->tgt_fov == nullptr))
            return fail(SMC_EINVAL, "frame %u: FOV masks must be given for the same volumes as the first pair", q + 1);
    }
    if ((st = c->check_sticky()) != SMC_OK) return st;
    if ((st = set_device(c)) != SMC_OK) return c->mark(st);
    for (smc_ctx *fr : c->frames) smc_destroy(fr);
    c->frames.clear();
    // each further pair is prepared by a context of its own (one particle,
    // one iteration: only its prepared volumes and launch settings are used)
    smc_params fp = c->p;
    fp.n_particles = 1;
    fp.n_iters = 1;
    for (uint32_t q = 0; q < n_extra; ++q) {
        smc_ctx *fr = nullptr;
        if ((st = smc_init(&fr, &src_frames[q], &tgt_frames[q], &fp, c->stream)) != SMC_OK) {
            const std::string msg = g_err;
            for (smc_ctx *g : c->frames) smc_destroy(g);
            c->frames.clear();
            pool_frame_constants(c);
            return fail(st, "frame %u: %s", q + 1, msg.c_str());
        }
        c->frames.push_back(fr);
        fr->items_np = c->f.n + 1;  // it scores this context's particles
        if ((st = smc_set_tuning(fr, c->layout, c->pt, c->zchunk)) != SMC_OK) return c->mark(st);
    }
    pool_frame_constants(c);
    return SMC_OK;
}

smc_status smc_set_tuning(smc_ctx *c, int32_t layout, int32_t pt, int32_t tile_depth) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    if (tile_depth == 0 || tile_depth > 256) return fail(SMC_EINVAL, "tile_depth must be in 1..256");
    if (layout >= kLayouts) return fail(SMC_EINVAL, "unknown layout %d", layout);
    if (pt >= 0 && !score_pt_supported(pt)) return fail(SMC_EINVAL, "particles_per_group must be 4, 8 or 16");
    smc_status st;
    if ((st = c->check_sticky()) != SMC_OK) return st;
    if ((st = set_device(c)) != SMC_OK) return c->mark(st);
    {
        // refuse a tuning whose launches would not fit one grid, leaving the context as it was
        const int old_pt = c->pt, old_z = c->zchunk;
        if (pt >= 0) c->pt = pt;
        if (tile_depth > 0) c->zchunk = tile_depth;
        st = check_items(c);
        c->pt = old_pt;
        c->zchunk = old_z;
        if (st != SMC_OK) return st;
    }
    if (layout >= 0) {
        if (c->mode == kModeImageTrilinear && !layout_fits(layout, c->sn))
            return fail(SMC_EINVAL, "layout %d cannot address a %d x %d x %d source (packed size >= 4 GiB or "
                        "a packed slice >= 16 MiB); use layout 0", layout, c->sn[0], c->sn[1], c->sn[2]);
        if ((st = prepare_layout(c, layout)) != SMC_OK) return c->mark(st);
        c->layout = layout;
    }
    for (smc_ctx *fr : c->frames)
        if ((st = smc_set_tuning(fr, layout, pt, tile_depth)) != SMC_OK) return c->mark(st);
    if (pt >= 0) c->pt = pt;
    if (tile_depth > 0) c->zchunk = tile_depth;
    if ((st = ensure_items(c)) != SMC_OK) return c->mark(st);
    return SMC_OK;
}

namespace {
struct TuneKey {
    int mode, score;
    int32_t sn[3], tn[3];
    bool sok, tfov;
    uint32_t n;
    bool operator<(const TuneKey &o) const {
        return std::memcmp(this, &o, sizeof(TuneKey)) < 0;
    }
};
struct TuneVal {
    int layout, pt, zchunk;
    double ms;
};
std::map<TuneKey, TuneVal> &tune_cache() {
    static std::map<TuneKey, TuneVal> m;
    return m;
}
std::mutex &tune_mutex() {
    static std::mutex m;
    return m;
}
}  // namespace

smc_status smc_autotune(smc_ctx *c, uint32_t reps, double *best_ms) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    if (reps < 1 || reps > 100) return fail(SMC_EINVAL, "reps must be in 1..100");
    smc_status st;
    if ((st = c->check_sticky()) != SMC_OK) return st;
    if ((st = set_device(c)) != SMC_OK) return c->mark(st);
    TuneKey key;
    std::memset(&key, 0, sizeof key);
    key.mode = c->mode;
    key.score = c->p.score;
    for (int d = 0; d < 3; ++d) {
        key.sn[d] = c->sn[d];
        key.tn[d] = c->tn[d];
    }
    key.sok = c->src_ok != nullptr;
    key.tfov = c->tgt_fov != nullptr;
    key.n = c->f.n;
    {
        std::lock_guard<std::mutex> g(tune_mutex());
        auto it = tune_cache().find(key);
        if (it != tune_cache().end()) {
            if ((st = smc_set_tuning(c, it->second.layout, it->second.pt, it->second.zchunk)) != SMC_OK) return st;
            if (best_ms) *best_ms = it->second.ms;
            return SMC_OK;
        }
    }
    const uint32_t np = c->f.n + 1;
    if ((st = ensure_eval(c, np)) != SMC_OK) return c->mark(st);
    // Two particle sets are timed: the prior (the context's current set,
    // spread over the whole limits box) and a concentrated cloud like the one
    // the filter evaluates after its first iterations (x0 +- 5 % of the
    // limits, a low-discrepancy fill), weighted by how often each occurs in a
    // registration: the cloud's locality decides which layout gathers best.
    {
        std::vector<double> xs(6ull * np);
        for (uint32_t i = 0; i < np; ++i)
            for (int d = 0; d < 6; ++d) {
                const double alpha = sqrt((double)(2 + 3 * d)) - floor(sqrt((double)(2 + 3 * d)));
                const double h = 0.5 + (double)i * alpha;
                xs[6ull * i + d] = c->p.x0[d] + 0.05 * c->p.limit[d] * (2.0 * (h - floor(h)) - 1.0);
            }
        if (hipMemcpyAsync(c->x_eval, xs.data(), 48ull * np, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
            launch_words(c->x_eval, np, c->f.geom, c->f.nearest, c->w_eval, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            return c->mark(fail(SMC_EDEVICE, "autotune particle set failed"));
    }
    const double w_conc = c->f.n_iters > 1 ? (double)(c->f.n_iters - 1) : 0.0;
    std::vector<int> layouts = {kLayoutRaw};
    if (c->mode == kModeImageTrilinear)
        layouts = {kLayoutRaw, kLayoutPairX, kLayoutQuadXY, kLayoutOct, kLayoutOctTile, kLayoutLerp};
    const int depths_img[] = {32, 256}, depths_mask[] = {16, 32, 256};
    const int *depths = c->mode == kModeMask ? depths_mask : depths_img;
    const int nd = c->mode == kModeMask ? 3 : 2;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    TuneVal best{c->layout, c->pt, c->zchunk, 1e30};
    smc_status result = SMC_OK;
    for (int lay : layouts)
        for (int pt : {4, 8})
            for (int q = 0; q < nd && result == SMC_OK && layout_fits(lay, c->sn); ++q) {
                if ((result = smc_set_tuning(c, lay, pt, depths[q])) != SMC_OK) break;
                double cost = 0.0;
                for (int set = 0; set < 2 && result == SMC_OK; ++set) {
                    // (the prior set is scored as smc_step's first iteration would score it)
                    ScoreLaunch L = c->score_launch(set == 0 ? c->f.words : c->w_eval, c->s_eval, 0, np, true,
                                                    set == 0 && c->prior_dispersed && c->k_done == 0);
                    if (c->p.score == SMC_SCORE_MI) L.hist = c->hist_eval;
                    double best_t = 1e30;  // the fastest of reps launches: robust to interference
                    for (uint32_t r = 0; r <= reps && result == SMC_OK; ++r) {
                        float ms = 0.0f;
                        if (launch_fill_u64(c->s_eval, 6ull * np, c->stream) != hipSuccess ||
                            hipEventRecord(e0, c->stream) != hipSuccess || launch_score(L, c->stream) != hipSuccess ||
                            hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                            result = fail(SMC_EDEVICE, "autotune launch failed");
                        if (r > 0) best_t = std::min(best_t, (double)ms);  // the first launch warms caches
                    }
                    cost += (set == 0 ? 1.0 : w_conc) * best_t;
                }
                const double avg = cost / (1.0 + w_conc);  // per launch over a registration
                if (avg < best.ms) best = TuneVal{lay, pt, depths[q], avg};
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the timed launches left counts in the evaluation histograms
    if (result == SMC_OK && c->hist_eval &&
        launch_fill_u64((unsigned long long *)c->hist_eval, (uint64_t)kMiBins * kMiBins * c->eval_cap / 2,
                        c->stream) != hipSuccess)
        result = fail(SMC_EDEVICE, "histogram clear failed");
    if (result != SMC_OK) return c->mark(result);
    if ((st = smc_set_tuning(c, best.layout, best.pt, best.zchunk)) != SMC_OK) return st;
    {
        std::lock_guard<std::mutex> g(tune_mutex());
        tune_cache()[key] = best;
    }
    if (best_ms) *best_ms = best.ms;
    return SMC_OK;
}

smc_status smc_get_tuning(smc_ctx *c, int32_t *layout, int32_t *pt, int32_t *tile_depth) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    if (layout) *layout = c->layout;
    if (pt) *pt = c->pt;
    if (tile_depth) *tile_depth = c->zchunk;
    return SMC_OK;
}

smc_status smc_profile(smc_ctx *c, int32_t enable) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    c->profiling = enable != 0;
    return SMC_OK;
}

smc_status smc_profile_read(smc_ctx *c, double *score_ms, uint64_t *score_n, double *filter_ms,
                            uint64_t *filter_n) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    smc_status st;
    if ((st = set_device(c)) != SMC_OK) return st;
    HIP_TRY(hipStreamSynchronize(c->stream));
    double sums[2] = {0.0, 0.0};
    uint64_t counts[2] = {0, 0};
    std::vector<std::pair<hipEvent_t, hipEvent_t>> *logs[2] = {&c->ev_score, &c->ev_filter};
    for (int q = 0; q < 2; ++q) {
        for (auto &pr : *logs[q]) {
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
            sums[q] += ms;
            counts[q] += 1;
            c->ev_pool.push_back(pr.first);
            c->ev_pool.push_back(pr.second);
        }
        logs[q]->clear();
    }
    if (score_ms) *score_ms = sums[0];
    if (score_n) *score_n = counts[0];
    if (filter_ms) *filter_ms = sums[1];
    if (filter_n) *filter_n = counts[1];
    return SMC_OK;
}

smc_status smc_profile_work(smc_ctx *c, uint64_t *evaluated, uint64_t *covered, uint64_t *interior) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    smc_status st;
    if ((st = set_device(c)) != SMC_OK) return st;
    std::vector<unsigned long long> w(kWorkSlots * kWorkSlotWords, 0ull);
    if (c->work) {
        HIP_TRY(hipMemcpyAsync(w.data(), c->work, w.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                               c->stream));
        HIP_TRY(launch_fill_u64(c->work, kWorkSlots * kWorkSlotWords, c->stream));
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    uint64_t ev = 0, cov = 0, in = 0;
    for (uint32_t q = 0; q < kWorkSlots; ++q) {
        ev += w[q * kWorkSlotWords];
        cov += w[q * kWorkSlotWords + 1];
        in += w[q * kWorkSlotWords + 2];
    }
    if (evaluated) *evaluated = ev;
    if (covered) *covered = cov;
    if (interior) *interior = in;
    return SMC_OK;
}

void smc_destroy(smc_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (smc_ctx *fr : c->frames) smc_destroy(fr);
    for (void *ptr : c->allocs) (void)hipFree(ptr);
    for (auto *log : {&c->ev_score, &c->ev_filter})
        for (auto &pr : *log) {
            c->ev_pool.push_back(pr.first);
            c->ev_pool.push_back(pr.second);
        }
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
}

smc_status warp_apply(const smc_volume *src, const double mat3x4[12], int32_t interp, uint8_t *dst, int32_t nx,
                      int32_t ny, int32_t nz, double sx, double sy, double sz, uint32_t n_frames,
                      int64_t src_frame_stride, int64_t dst_frame_stride, void *hip_stream) {
    g_err.clear();
    smc_status st;
    if ((st = check_volume(src, "src")) != SMC_OK) return st;
    if (!mat3x4 || !dst) return fail(SMC_EINVAL, "mat3x4 and dst must not be NULL");
    for (int q = 0; q < 12; ++q)
        if (!isfinite(mat3x4[q])) return fail(SMC_EINVAL, "matrix entry %d is not finite", q);
    if (interp != SMC_INTERP_NEAREST && interp != SMC_INTERP_TRILINEAR)
        return fail(SMC_EINVAL, "unknown interpolation %d", interp);
    if (nx < 1 || ny < 1 || nz < 1 || nx > 65535 || ny > 65535 || nz > 65535)
        return fail(SMC_EINVAL, "output dimensions out of range");
    if (!(sx > 0 && sy > 0 && sz > 0)) return fail(SMC_EINVAL, "output spacing must be positive");
    if (n_frames < 1 || n_frames > 65535) return fail(SMC_EINVAL, "n_frames must be in 1..65535");
    const int64_t vs = (int64_t)src->nx * src->ny * src->nz, vt = (int64_t)nx * ny * nz;
    if (vt >= ((int64_t)1 << 31)) return fail(SMC_EINVAL, "output frames of 2^31 voxels or more");
    if (n_frames > 1 && (src_frame_stride < vs || dst_frame_stride < vt))
        return fail(SMC_EINVAL, "frame strides smaller than a frame");
    const double ts[3] = {sx, sy, sz}, ss[3] = {src->sx, src->sy, src->sz};
    float w[12];
    words_from_matrix(mat3x4, ts, ss, interp == SMC_INTERP_NEAREST, w);
    const int32_t sn[3] = {src->nx, src->ny, src->nz}, tn[3] = {nx, ny, nz};
    hipError_t e = launch_warp_apply(src->data, sn, w, interp == SMC_INTERP_TRILINEAR, dst, tn, n_frames,
                                     src_frame_stride, dst_frame_stride, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(SMC_EDEVICE, "warp_apply launch failed: %s", hipGetErrorString(e));
    return SMC_OK;
}

}  // extern "C"

// ===================================================================== batches

struct smc_batch {
    hipStream_t stream = nullptr;
    std::vector<smc_ctx *> pairs;
    std::vector<FilterState> states;
    FilterState *states_dev = nullptr;
    uint32_t kmax_all = 0, max_threads = 0;
    struct Class {
        BatchPlan plan{};
        // the first iteration over uniform priors (image classes whose pairs
        // all score a dispersed prior from one other layout): same items,
        // arguments for that layout
        BatchPlan plan_first{};
        bool has_first = false;
        void *fargs = nullptr;
        std::vector<uint32_t> members;
        void *args = nullptr;
        uint32_t *offs = nullptr, *kmax = nullptr, *lists = nullptr;
    } cls[4];  // 0 masks; 1, 2, 3 trilinear images by source FOV validity mode 0, 1, 2
    std::vector<uint32_t> images;   // all trilinear image pairs
    std::vector<uint32_t> singles;  // pairs outside the classes (nearest-neighbour images) run per pair
    std::vector<void *> allocs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipStream_t caller = nullptr;

    template <typename T>
    smc_status alloc(T **out, size_t count) {
        void *ptr = nullptr;
        if (hipMalloc(&ptr, count * sizeof(T) > 0 ? count * sizeof(T) : 1) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SMC_ENOMEM, "hipMalloc failed in smc_batch_init");
        }
        allocs.push_back(ptr);
        *out = static_cast<T *>(ptr);
        return SMC_OK;
    }
};

namespace {

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        cus = 256;
    return cus;
}

// Work list of one class.  A pair's items run tile by tile with the
// particle groups fastest; each pair is cut into eight contiguous ranges of
// items, range x going to XCD x, so every XCD sweeps one eighth of each
// volume (its L2 holds that part of the source instead of a whole large
// volume) and the lists stay balanced whatever the mix of pairs.
smc_status plan_class(smc_batch *b, smc_batch::Class &C, int mode, int vmode) {
    const uint32_t n = (uint32_t)C.members.size();
    C.has_first = false;
    if (n == 0) {
        C.plan = BatchPlan{};  // an empty class launches nothing (also after a re-plan)
        return SMC_OK;
    }
    const size_t ab = score_args_bytes();
    std::vector<uint8_t> args(ab * n);
    std::vector<uint32_t> offs(n + 1, 0), kmax(n);
    std::vector<double> work(n);
    int pt = 8, layout = kLayoutRaw;
    for (uint32_t q = 0; q < n; ++q) {
        smc_ctx *c = b->pairs[C.members[q]];
        ScoreLaunch L = c->score_launch(c->f.words, c->f.sums, 0, c->f.n + 1, true);
        // the persistent mask launch reads every pair's source bitmap
        if (mode == kModeMask && !L.src_bits) return fail(SMC_EINVAL, "mask pair %u has no source bitmap", C.members[q]);
        if (q == 0) {
            pt = L.pt;
            layout = L.layout;
        } else if (L.pt != pt || L.layout != layout) {
            return fail(SMC_EINVAL, "batch class mixes tunings (pair %u)", C.members[q]);
        }
        score_args(L, args.data() + ab * q);
        const uint32_t items = score_items(L);
        offs[q + 1] = offs[q] + items;
        kmax[q] = c->f.n_iters;
        work[q] = (double)items * (double)c->tn[2];
    }
    // largest pairs first, so the longest runs start early on every XCD
    std::vector<uint32_t> order(n);
    for (uint32_t q = 0; q < n; ++q) order[q] = q;
    std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t c) { return work[a] > work[c]; });
    std::vector<std::vector<uint32_t>> lists(8);
    for (uint32_t q : order) {
        const uint32_t items = offs[q + 1] - offs[q];
        for (uint32_t x = 0; x < 8; ++x) {
            const uint32_t lo = offs[q] + (uint32_t)((uint64_t)items * x / 8);
            const uint32_t hi = offs[q] + (uint32_t)((uint64_t)items * (x + 1) / 8);
            for (uint32_t g = lo; g < hi; ++g) lists[x].push_back(g);
        }
    }
    std::vector<uint32_t> flat;
    C.plan.list_off[0] = 0;
    for (int x = 0; x < 8; ++x) {
        flat.insert(flat.end(), lists[x].begin(), lists[x].end());
        C.plan.list_off[x + 1] = (uint32_t)flat.size();
    }
    smc_status st;
    if ((st = b->alloc((uint8_t **)&C.args, args.size())) != SMC_OK || (st = b->alloc(&C.offs, n + 1)) != SMC_OK ||
        (st = b->alloc(&C.kmax, n)) != SMC_OK || (st = b->alloc(&C.lists, flat.size())) != SMC_OK ||
        (st = b->alloc(&C.plan.counters, 8ull * std::max(1u, b->kmax_all))) != SMC_OK)
        return st;
    if (mode == kModeMask) {
        // live item lists of the cull pre-pass (one list buffer, counts per iteration)
        uint2 *live = nullptr;
        uint32_t *lc = nullptr;
        if ((st = b->alloc(&live, std::max<size_t>(1, flat.size()))) != SMC_OK ||
            (st = b->alloc(&lc, (size_t)(kItemCounterWords / 2) * std::max(1u, b->kmax_all))) != SMC_OK)
            return st;
        C.plan.live = live;
        C.plan.live_counts = lc;
    }
    HIP_TRY(hipMemcpy(C.args, args.data(), args.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(C.offs, offs.data(), 4 * (n + 1), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(C.kmax, kmax.data(), 4 * n, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(C.lists, flat.data(), 4 * flat.size(), hipMemcpyHostToDevice));
    C.plan.mode = mode;
    C.plan.layout = layout;
    C.plan.pt = pt;
    C.plan.vmode = vmode;
    C.plan.pairs = C.args;
    C.plan.offs = C.offs;
    C.plan.kmax = C.kmax;
    C.plan.lists = C.lists;
    C.plan.n_pairs = n;
    // persistent grid: as many workgroups as stay resident, a multiple of the 8 XCDs
    const uint32_t per_cu = (uint32_t)batch_blocks_per_cu(C.plan);
    C.plan.grid = 8 * (((uint32_t)device_cus() * per_cu + 7) / 8);
    if (mode == kModeImageTrilinear) {
        // a first-iteration plan when every pair scores its uniform prior from
        // the same other layout with the same items and FOV mode
        std::vector<uint8_t> fargs(ab * n);
        bool ok = true;
        int flayout = -1;
        for (uint32_t q = 0; q < n && ok; ++q) {
            const smc_ctx *c = b->pairs[C.members[q]];
            const ScoreLaunch F = c->score_launch(c->f.words, c->f.sums, 0, c->f.n + 1, true, true);
            if (q == 0) flayout = F.layout;
            ok = !c->f.has_proposal && F.layout == flayout && F.layout != layout && F.pt == pt &&
                 score_vmode(F) == vmode && score_items(F) == offs[q + 1] - offs[q];
            if (ok) score_args(F, fargs.data() + ab * q);
        }
        if (ok) {
            if ((st = b->alloc((uint8_t **)&C.fargs, fargs.size())) != SMC_OK) return st;
            HIP_TRY(hipMemcpy(C.fargs, fargs.data(), fargs.size(), hipMemcpyHostToDevice));
            C.plan_first = C.plan;
            C.plan_first.layout = flayout;
            C.plan_first.pairs = C.fargs;
            const uint32_t fper = (uint32_t)batch_blocks_per_cu(C.plan_first);
            C.plan_first.grid = 8 * (((uint32_t)device_cus() * fper + 7) / 8);
            C.has_first = true;
        }
    }
    return SMC_OK;
}

// Split the image pairs by source FOV validity mode (one kernel variant per
// class keeps each variant's register budget) and plan every class.
smc_status plan_all(smc_batch *b) {
    // one kernel variant serves a class: every image pair takes the first
    // image pair's layout and particles per group, every mask pair the first
    // mask pair's particles per group (before the FOV modes are read, since a
    // layout decides whether a pair has an in-band FOV sentinel)
    for (int q = 0; q < 2; ++q) {
        const std::vector<uint32_t> &members = q == 0 ? b->cls[0].members : b->images;
        if (members.empty()) continue;
        const smc_ctx *c0 = b->pairs[members[0]];
        for (uint32_t i : members) {
            smc_ctx *c = b->pairs[i];
            if ((q == 1 && c->layout != c0->layout) || c->pt != c0->pt)
                if (smc_set_tuning(c, q == 1 ? c0->layout : -1, c0->pt, -1) != SMC_OK)
                    return fail(SMC_EINVAL, "pair %u cannot take the tuning of pair %u", i, members[0]);
        }
    }
    for (int q = 1; q < 4; ++q) b->cls[q].members.clear();
    for (uint32_t i : b->images) {
        smc_ctx *c = b->pairs[i];
        const int vm = score_vmode(c->score_launch(c->f.words, c->f.sums, 0, c->f.n + 1, true));
        b->cls[1 + vm].members.push_back(i);
    }
    smc_status st;
    for (int q = 0; q < 4; ++q)
        if ((st = plan_class(b, b->cls[q], q == 0 ? kModeMask : kModeImageTrilinear, q == 0 ? 0 : q - 1)) != SMC_OK)
            return st;
    return SMC_OK;
}

// The whole batched run, recorded on b->stream (captured into the graph).
smc_status record_run(smc_batch *b) {
    HIP_TRY(launch_init_batch(b->states_dev, (uint32_t)b->pairs.size(), b->max_threads, b->stream));
    for (smc_ctx *c : b->pairs) HIP_TRY(launch_fill_u64(c->f.sums, 6ull * (c->f.n + 1), b->stream));
    // the item queues start empty on every run (a fill kernel, so graph replays clear them too)
    for (int q = 0; q < 4; ++q)
        if (b->cls[q].plan.n_pairs)
            HIP_TRY(launch_fill_u64((unsigned long long *)b->cls[q].plan.counters, 4ull * std::max(1u, b->kmax_all),
                                    b->stream));
    if (b->cls[0].plan.n_pairs && b->cls[0].plan.live_counts)
        HIP_TRY(launch_fill_u64((unsigned long long *)b->cls[0].plan.live_counts,
                                (uint64_t)(kItemCounterWords / 4) * std::max(1u, b->kmax_all), b->stream));
    for (uint32_t k = 1; k <= b->kmax_all; ++k) {
        for (int q = 0; q < 4; ++q) {
            const smc_batch::Class &C = b->cls[q];
            HIP_TRY(launch_batch_score(k == 1 && C.has_first ? C.plan_first : C.plan, k, b->stream));
        }
        for (uint32_t i : b->singles) {
            smc_ctx *c = b->pairs[i];
            if (k <= c->f.n_iters) HIP_TRY(launch_score_frames(c, c->f.words, c->f.sums, c->hist, 0, c->f.n + 1, true));
        }
        HIP_TRY(launch_filter_batch(b->states_dev, (uint32_t)b->pairs.size(), k, b->stream));
        for (smc_ctx *c : b->pairs)
            if (c->f.n_iters == k) {
                HIP_TRY(launch_score_frames(c, c->f.words, c->f.sums, c->hist, c->f.n, 1, true));
                HIP_TRY(launch_ghost_final(c->f, b->stream));
            }
    }
    return SMC_OK;
}

}  // namespace

extern "C" {

smc_status smc_batch_init(smc_batch **out, uint32_t n_pairs, const smc_volume *src, const smc_volume *tgt,
                          const smc_params *p, void *hip_stream) {
    g_err.clear();
    if (!out) return fail(SMC_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_pairs < 1 || n_pairs > 4096) return fail(SMC_EINVAL, "n_pairs must be in 1..4096");
    if (!src || !tgt || !p) return fail(SMC_EINVAL, "src, tgt and p must not be NULL");
    smc_batch *b = new (std::nothrow) smc_batch();
    if (!b) return fail(SMC_ENOMEM, "host allocation failed");
    b->caller = (hipStream_t)hip_stream;
    auto bail = [&](smc_status st) {
        std::string msg = g_err;
        smc_batch_destroy(b);
        g_err = msg;
        return st;
    };
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess)
        return bail(fail(SMC_EDEVICE, "stream / event creation failed"));
    smc_status st;
    for (uint32_t i = 0; i < n_pairs; ++i) {
        smc_ctx *c = nullptr;
        if ((st = smc_init(&c, &src[i], &tgt[i], &p[i], b->stream)) != SMC_OK) {
            std::string msg = g_err;
            return bail(fail(st, "pair %u: %s", i, msg.c_str()));
        }
        c->in_batch = true;
        b->pairs.push_back(c);
        b->states.push_back(c->f);
        b->kmax_all = std::max(b->kmax_all, c->f.n_iters);
        b->max_threads = std::max(b->max_threads, std::max(c->f.n, c->f.n_iters + 1));
        if (c->mode == kModeMask) b->cls[0].members.push_back(i);
        else if (c->mode == kModeImageTrilinear && c->p.score != SMC_SCORE_MI) b->images.push_back(i);
        else b->singles.push_back(i);
    }
    // one layout / particles-per-group for all trilinear pairs: the first pair's
    for (uint32_t q = 1; q < b->images.size(); ++q) {
        smc_ctx *c0 = b->pairs[b->images[0]], *c = b->pairs[b->images[q]];
        if ((st = smc_set_tuning(c, c0->layout, c0->pt, c0->zchunk)) != SMC_OK) return bail(st);
    }
    if ((st = b->alloc(&b->states_dev, n_pairs)) != SMC_OK) return bail(st);
    if (hipMemcpy(b->states_dev, b->states.data(), sizeof(FilterState) * n_pairs, hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(SMC_EDEVICE, "upload of filter states failed"));
    if ((st = plan_all(b)) != SMC_OK) return bail(st);
    if (hipStreamSynchronize(b->stream) != hipSuccess) return bail(fail(SMC_EDEVICE, "batch preparation failed"));
    *out = b;
    return SMC_OK;
}

smc_status smc_batch_set_seeds(smc_batch *b, const uint64_t *seeds) {
    if (!b) return fail(SMC_EINVAL, "batch is NULL");
    if (!seeds) return SMC_OK;
    for (size_t i = 0; i < b->pairs.size(); ++i) {
        b->states[i].seed = seeds[i];
        b->pairs[i]->f.seed = seeds[i];
        b->pairs[i]->p.seed = seeds[i];
    }
    // ordered on the batch stream, so it cannot overtake a running replay
    HIP_TRY(hipMemcpyAsync(b->states_dev, b->states.data(), sizeof(FilterState) * b->states.size(),
                           hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return SMC_OK;
}

smc_status smc_batch_run(smc_batch *b) {
    if (!b) return fail(SMC_EINVAL, "batch is NULL");
    for (smc_ctx *c : b->pairs) {
        smc_status st = c->check_sticky();
        if (st != SMC_OK) return st;
    }
    if (!b->exec) {
        HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        smc_status st = record_run(b);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(b->stream, &g);
        if (st != SMC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return fail(SMC_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
        b->graph = g;
        HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    HIP_TRY(hipEventRecord(b->ev_in, b->caller));
    HIP_TRY(hipStreamWaitEvent(b->stream, b->ev_in, 0));
    HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    HIP_TRY(hipEventRecord(b->ev_out, b->stream));
    HIP_TRY(hipStreamWaitEvent(b->caller, b->ev_out, 0));
    for (smc_ctx *c : b->pairs) c->k_done = c->f.n_iters;
    return SMC_OK;
}

smc_status smc_batch_autotune(smc_batch *b, uint32_t reps) {
    if (!b) return fail(SMC_EINVAL, "batch is NULL");
    smc_status st;
    for (int q = 0; q < 2; ++q) {
        const std::vector<uint32_t> &members = q == 0 ? b->cls[0].members : b->images;
        if (members.empty()) continue;
        uint32_t big = members[0];
        double work = 0.0;
        for (uint32_t i : members) {
            smc_ctx *c = b->pairs[i];
            const double w = (double)c->tn[0] * c->tn[1] * c->tn[2] * (double)(c->f.n + 1);
            if (w > work) {
                work = w;
                big = i;
            }
        }
        smc_ctx *c0 = b->pairs[big];
        if ((st = smc_autotune(c0, reps, nullptr)) != SMC_OK) return st;
        for (uint32_t i : members)
            if ((st = smc_set_tuning(b->pairs[i], c0->layout, c0->pt, c0->zchunk)) != SMC_OK) return st;
    }
    if ((st = plan_all(b)) != SMC_OK) return st;
    HIP_TRY(hipStreamSynchronize(b->stream));
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    return SMC_OK;
}

smc_ctx *smc_batch_pair(smc_batch *b, uint32_t i) {
    if (!b || i >= b->pairs.size()) return nullptr;
    return b->pairs[i];
}

void smc_batch_destroy(smc_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (smc_ctx *c : b->pairs) smc_destroy(c);
    for (void *ptr : b->allocs) (void)hipFree(ptr);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // extern "C"

// ===================================================================== learned proposal

struct smc_cnn {
    hipStream_t stream = nullptr;
    uint32_t max_batch = 0;
    CnnBuffers c{};
    uint16_t *input = nullptr;  // max_batch x 2 x 64^3 FP16
    float *out = nullptr, *target = nullptr, *loss = nullptr;
    int adam_t = 0;
    std::vector<void *> allocs;
    template <typename T>
    smc_status alloc(T **p, size_t count) {
        void *ptr = nullptr;
        if (hipMalloc(&ptr, count * sizeof(T) > 0 ? count * sizeof(T) : 1) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SMC_ENOMEM, "hipMalloc failed in smc_cnn_create");
        }
        allocs.push_back(ptr);
        *p = static_cast<T *>(ptr);
        return SMC_OK;
    }
};

extern "C" {

smc_status smc_cnn_create(smc_cnn **out, uint32_t max_batch, void *hip_stream) {
    g_err.clear();
    if (!out) return fail(SMC_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_batch < 1 || max_batch > 1024) return fail(SMC_EINVAL, "max_batch must be in 1..1024");
    smc_cnn *n = new (std::nothrow) smc_cnn();
    if (!n) return fail(SMC_ENOMEM, "host allocation failed");
    n->stream = (hipStream_t)hip_stream;
    n->max_batch = max_batch;
    CnnBuffers &c = n->c;
    c.n_params = cnn_param_offset(10);
    const size_t side3 = (size_t)kCnnSide * kCnnSide * kCnnSide;
    smc_status st;
    auto bail = [&](smc_status e) {
        smc_cnn_destroy(n);
        return e;
    };
    if ((st = n->alloc(&c.params, c.n_params)) != SMC_OK || (st = n->alloc(&c.grads, c.n_params)) != SMC_OK ||
        (st = n->alloc(&c.adam_m, c.n_params)) != SMC_OK || (st = n->alloc(&c.adam_v, c.n_params)) != SMC_OK ||
        (st = n->alloc(&c.wbf16, cnn_param_offset(8))) != SMC_OK ||
        (st = n->alloc(&n->input, 2 * side3 * max_batch)) != SMC_OK ||
        (st = n->alloc(&n->out, 12ull * max_batch)) != SMC_OK ||
        (st = n->alloc(&n->target, 12ull * max_batch)) != SMC_OK || (st = n->alloc(&n->loss, 4)) != SMC_OK ||
        (st = n->alloc(&c.dout, 12ull * max_batch)) != SMC_OK ||
        (st = n->alloc(&c.partial, (size_t)cnn_partial_floats((int)max_batch))) != SMC_OK)
        return bail(st);
    c.partial_cap = cnn_partial_floats((int)max_batch);
    for (int L = 0; L < 4; ++L) {
        const size_t d = (size_t)(kCnnSide >> (L + 1));
        const size_t elems = (size_t)max_batch * kCnnChannels[L + 1] * d * d * d;
        if ((st = n->alloc(&c.act[L], elems)) != SMC_OK || (st = n->alloc(&c.dact[L], elems)) != SMC_OK)
            return bail(st);
    }
    std::vector<float> zeros((size_t)c.n_params, 0.0f);
    if (hipMemcpy(c.params, zeros.data(), 4 * c.n_params, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c.adam_m, zeros.data(), 4 * c.n_params, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c.adam_v, zeros.data(), 4 * c.n_params, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c.grads, zeros.data(), 4 * c.n_params, hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(SMC_EDEVICE, "parameter initialisation failed"));
    if (cnn_refresh_bf16(c, n->stream) != hipSuccess || hipStreamSynchronize(n->stream) != hipSuccess)
        return bail(fail(SMC_EDEVICE, "parameter initialisation failed"));
    *out = n;
    return SMC_OK;
}

smc_status smc_cnn_set_params(smc_cnn *n, const float *host, size_t count) {
    if (!n || !host) return fail(SMC_EINVAL, "net and params must not be NULL");
    if (count != (size_t)n->c.n_params) return fail(SMC_EINVAL, "%zu parameters given, %lld expected", count,
                                                    (long long)n->c.n_params);
    for (size_t q = 0; q < count; ++q)
        if (!isfinite(host[q])) return fail(SMC_EINVAL, "parameter %zu is not finite", q);
    std::vector<float> zeros(count, 0.0f);
    HIP_TRY(hipMemcpyAsync(n->c.params, host, 4 * count, hipMemcpyHostToDevice, n->stream));
    HIP_TRY(hipMemcpyAsync(n->c.adam_m, zeros.data(), 4 * count, hipMemcpyHostToDevice, n->stream));
    HIP_TRY(hipMemcpyAsync(n->c.adam_v, zeros.data(), 4 * count, hipMemcpyHostToDevice, n->stream));
    HIP_TRY(cnn_refresh_bf16(n->c, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
    n->adam_t = 0;
    return SMC_OK;
}

smc_status smc_cnn_get_params(smc_cnn *n, float *host, size_t count) {
    if (!n || !host) return fail(SMC_EINVAL, "net and params must not be NULL");
    if (count != (size_t)n->c.n_params) return fail(SMC_EINVAL, "wrong parameter count");
    HIP_TRY(hipMemcpyAsync(host, n->c.params, 4 * count, hipMemcpyDeviceToHost, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
    return SMC_OK;
}

smc_status smc_cnn_input(smc_cnn *n, uint32_t slot, const smc_volume *src, const smc_volume *tgt, float scale) {
    if (!n) return fail(SMC_EINVAL, "net is NULL");
    if (slot >= n->max_batch) return fail(SMC_EINVAL, "slot %u beyond max_batch", slot);
    if (!isfinite(scale)) return fail(SMC_EINVAL, "scale must be finite");
    smc_status st;
    if ((st = check_volume(src, "src")) != SMC_OK || (st = check_volume(tgt, "tgt")) != SMC_OK) return st;
    const size_t side3 = (size_t)kCnnSide * kCnnSide * kCnnSide;
    const int32_t sn[3] = {src->nx, src->ny, src->nz}, tn[3] = {tgt->nx, tgt->ny, tgt->nz};
    HIP_TRY(cnn_downsample(src->data, sn, scale, n->input + 2 * side3 * slot, n->stream));
    HIP_TRY(cnn_downsample(tgt->data, tn, scale, n->input + 2 * side3 * slot + side3, n->stream));
    return SMC_OK;
}

smc_status smc_cnn_read_input(smc_cnn *n, uint32_t slot, uint16_t *host) {
    if (!n || !host) return fail(SMC_EINVAL, "net and host must not be NULL");
    if (slot >= n->max_batch) return fail(SMC_EINVAL, "slot %u beyond max_batch", slot);
    const size_t side3 = (size_t)kCnnSide * kCnnSide * kCnnSide;
    HIP_TRY(hipMemcpyAsync(host, n->input + 2 * side3 * slot, 4 * side3, hipMemcpyDeviceToHost, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
    return SMC_OK;
}

smc_status smc_cnn_forward(smc_cnn *n, uint32_t B, float *out_host) {
    if (!n || !out_host) return fail(SMC_EINVAL, "net and out must not be NULL");
    if (B < 1 || B > n->max_batch) return fail(SMC_EINVAL, "batch %u outside 1..%u", B, n->max_batch);
    HIP_TRY(cnn_forward(n->c, n->input, (int)B, n->out, n->stream));
    HIP_TRY(hipMemcpyAsync(out_host, n->out, 48ull * B, hipMemcpyDeviceToHost, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
    return SMC_OK;
}

smc_status smc_cnn_backward(smc_cnn *n, uint32_t B, const float *target_host, float *loss, float *grads_host) {
    if (!n || !target_host) return fail(SMC_EINVAL, "net and target must not be NULL");
    if (B < 1 || B > n->max_batch) return fail(SMC_EINVAL, "batch %u outside 1..%u", B, n->max_batch);
    for (size_t q = 0; q < 12ull * B; ++q)
        if (!isfinite(target_host[q]) || (q % 12 >= 6 && target_host[q] < 0.0f))
            return fail(SMC_EINVAL, "target %zu must be finite (variances non-negative)", q);
    HIP_TRY(hipMemcpyAsync(n->target, target_host, 48ull * B, hipMemcpyHostToDevice, n->stream));
    HIP_TRY(cnn_forward(n->c, n->input, (int)B, n->out, n->stream));
    HIP_TRY(cnn_backward(n->c, n->input, (int)B, n->out, n->target, n->loss, n->stream));
    float l = 0.0f;
    HIP_TRY(hipMemcpyAsync(&l, n->loss, 4, hipMemcpyDeviceToHost, n->stream));
    if (grads_host)
        HIP_TRY(hipMemcpyAsync(grads_host, n->c.grads, 4 * n->c.n_params, hipMemcpyDeviceToHost, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
    if (loss) *loss = l;
    return SMC_OK;
}

smc_status smc_cnn_step(smc_cnn *n, float lr) {
    if (!n) return fail(SMC_EINVAL, "net is NULL");
    if (!(lr > 0.0f) || !isfinite(lr)) return fail(SMC_EINVAL, "lr must be positive");
    n->adam_t += 1;
    HIP_TRY(cnn_adam(n->c, lr, n->adam_t, n->stream));
    return SMC_OK;
}

void smc_cnn_destroy(smc_cnn *n) {
    if (!n) return;
    (void)hipStreamSynchronize(n->stream);
    for (void *p : n->allocs) (void)hipFree(p);
    delete n;
}

smc_status smc_cloud_moments(smc_ctx *c, double var_floor, double mean[6], double var[6]) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    if (!mean || !var) return fail(SMC_EINVAL, "mean and var must not be NULL");
    if (!(var_floor >= 0.0) || !isfinite(var_floor)) return fail(SMC_EINVAL, "var_floor must be finite and >= 0");
    if (c->k_done == 0) return fail(SMC_ESTATE, "no iteration has run: the particles carry no weights yet");
    smc_status st;
    if ((st = c->check_sticky()) != SMC_OK) return st;
    if ((st = set_device(c)) != SMC_OK) return c->mark(st);
    if ((st = ensure_eval(c, 2)) != SMC_OK) return c->mark(st);
    double m[12];
    HIP_TRY(launch_cloud_moments(c->f, c->x_eval, c->stream));
    HIP_TRY(hipMemcpyAsync(m, c->x_eval, sizeof m, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    // in units of the limits about x0, as the network predicts them
    for (int d = 0; d < 6; ++d) {
        const double L = c->f.limit[d];
        mean[d] = (m[d] - c->f.x0[d]) / L;
        var[d] = fmax(m[6 + d] / (L * L), var_floor);
    }
    return SMC_OK;
}

smc_status smc_set_proposal_from_network(smc_ctx *c, const float out[12], double var_scale, double mean_out[6],
                                         double logvar_out[6]) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    if (!out) return fail(SMC_EINVAL, "out is NULL");
    if (!(var_scale > 0.0) || !isfinite(var_scale)) return fail(SMC_EINVAL, "var_scale must be finite and positive");
    for (int q = 0; q < 12; ++q)
        if (!isfinite(out[q])) return fail(SMC_EINVAL, "network output %d is not finite", q);
    double mean[6], logvar[6];
    for (int d = 0; d < 6; ++d) {
        const double L = c->f.limit[d];
        const double u = fmin(fmax((double)out[d], -1.0), 1.0);
        const double l = fmin(fmax((double)out[6 + d], -20.0), 2.0);
        mean[d] = c->f.x0[d] + u * L;
        logvar[d] = l + 2.0 * log(L) + log(var_scale);
    }
    const smc_status st = smc_set_proposal(c, mean, logvar);
    if (st != SMC_OK) return st;
    if (mean_out) memcpy(mean_out, mean, sizeof mean);
    if (logvar_out) memcpy(logvar_out, logvar, sizeof logvar);
    return SMC_OK;
}

smc_status smc_set_proposal(smc_ctx *c, const double mean[6], const double logvar[6]) {
    if (!c) return fail(SMC_EINVAL, "ctx is NULL");
    if (!mean) {
        c->f.has_proposal = 0;
        return SMC_OK;
    }
    if (!logvar) return fail(SMC_EINVAL, "logvar is NULL");
    if (!finite6(mean) || !finite6(logvar)) return fail(SMC_EINVAL, "proposal must be finite");
    for (int d = 0; d < 6; ++d)
        if (logvar[d] < -60.0 || logvar[d] > 60.0) return fail(SMC_EINVAL, "logvar[%d] out of range", d);
    if (!c->f.lq) {
        smc_status st = c->alloc(&c->f.lq, c->f.n);
        if (st != SMC_OK) return st;
    }
    c->f.has_proposal = 1;
    for (int d = 0; d < 6; ++d) {
        c->f.prop_mu[d] = mean[d];
        c->f.prop_sigma[d] = exp(0.5 * logvar[d]);
    }
    return SMC_OK;
}

}  // extern "C"
