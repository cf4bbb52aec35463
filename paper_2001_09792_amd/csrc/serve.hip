// serve.hip -- admission pool and the continuous-batching render engine.
//
// The paper's renderer is a request loop: frames of different scenes are
// dispatched one after another, and its resource manager keeps loaded
// resources for reuse (section 2.2).  Here many frames share the device at
// once.  The engine runs the breadth-first Whitted loop as a sequence of
// passes; each pass traces, shades and shadows the queued rays of every
// frame in flight, whatever its recursion depth.  A frame admitted between
// passes queues its camera rays for the next pass and leaves after the pass
// at its own depth limit, so frames join and leave while others are
// mid-flight.  Admission reserves, per frame, the queue entries a pass can
// hold for it at worst and a contiguous range of pixel accumulators; the
// caller sizes the whole engine (queues, accumulators, tables) from its
// memory budget.
#include <algorithm>
#include <cstring>
#include <iterator>
#include <map>
#include <new>
#include <set>
#include <vector>

#include "wavefront.h"

// ------------------------------------------------------------ pool
struct rg_pool {
    int64_t max_rays = 0, max_pixels = 0;
    int32_t max_jobs = 0;
    int64_t rays_used = 0, pixels_used = 0;
    int32_t jobs_used = 0;
    std::map<int64_t, int64_t> free_px;  // offset -> length, disjoint, coalesced
    std::set<int32_t> free_slots;
    std::vector<int64_t> slot_rays, slot_off, slot_pix;
};

namespace {

bool pool_init(rg_pool &p, int64_t max_rays, int64_t max_pixels, int32_t max_jobs) {
    if (max_rays < 1 || max_rays > (1ll << 31) || max_pixels < 1 || max_pixels > (1ll << 31) || max_jobs < 1 ||
        max_jobs > (1 << 20))
        return false;
    p.max_rays = max_rays;
    p.max_pixels = max_pixels;
    p.max_jobs = max_jobs;
    p.free_px[0] = max_pixels;
    for (int32_t s = 0; s < max_jobs; ++s) p.free_slots.insert(s);
    p.slot_rays.assign((size_t)max_jobs, -1);
    p.slot_off.assign((size_t)max_jobs, -1);
    p.slot_pix.assign((size_t)max_jobs, 0);
    return true;
}

// *slot = -1 when the request does not fit now; RG_ERR_OUT_OF_MEMORY when it
// would not fit an empty pool either.
rg_status pool_reserve(rg_pool &p, int64_t rays, int64_t pixels, int32_t *slot, int64_t *pix_off) {
    *slot = -1;
    *pix_off = -1;
    if (rays < 1 || pixels < 1) return RG_ERR_INVALID_ARG;
    if (rays > p.max_rays || pixels > p.max_pixels) return RG_ERR_OUT_OF_MEMORY;
    if (p.free_slots.empty() || p.rays_used + rays > p.max_rays) return RG_OK;
    auto it = p.free_px.begin();
    for (; it != p.free_px.end(); ++it)
        if (it->second >= pixels) break;
    if (it == p.free_px.end()) return RG_OK;
    const int64_t off = it->first, len = it->second;
    p.free_px.erase(it);
    if (len > pixels) p.free_px[off + pixels] = len - pixels;
    const int32_t s = *p.free_slots.begin();
    p.free_slots.erase(p.free_slots.begin());
    p.slot_rays[s] = rays;
    p.slot_off[s] = off;
    p.slot_pix[s] = pixels;
    p.rays_used += rays;
    p.pixels_used += pixels;
    p.jobs_used += 1;
    *slot = s;
    *pix_off = off;
    return RG_OK;
}

rg_status pool_release(rg_pool &p, int32_t s) {
    if (s < 0 || s >= p.max_jobs || p.slot_rays[s] < 0) return RG_ERR_INVALID_ARG;
    int64_t off = p.slot_off[s], len = p.slot_pix[s];
    auto next = p.free_px.lower_bound(off);
    if (next != p.free_px.end() && next->first == off + len) {
        len += next->second;
        next = p.free_px.erase(next);
    }
    if (next != p.free_px.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == off) {
            off = prev->first;
            len += prev->second;
            p.free_px.erase(prev);
        }
    }
    p.free_px[off] = len;
    p.rays_used -= p.slot_rays[s];
    p.pixels_used -= p.slot_pix[s];
    p.jobs_used -= 1;
    p.slot_rays[s] = -1;
    p.slot_off[s] = -1;
    p.slot_pix[s] = 0;
    p.free_slots.insert(s);
    return RG_OK;
}

// Queue entries one pass can hold for a frame, at worst: a glass hit spawns
// a reflection and a refraction child, a mirror hit one child, a diffuse
// hit none; a pass at depth k therefore holds at most pixels * 2^k entries
// of the frame with glass, pixels without.
rg_status reservation(const rg_job *J, int64_t *rays, int64_t *pixels, int32_t *growth) {
    if (!J || !J->mats || J->n_mats < 1 || J->width < 1 || J->height < 1 || J->max_depth < 0 ||
        J->max_depth > RG_MAX_DEPTH)
        return RG_ERR_INVALID_ARG;
    const int64_t pix = (int64_t)J->width * J->height;
    if (pix > (1ll << 31)) return RG_ERR_UNSUPPORTED;
    bool glass = false;
    for (int32_t m = 0; m < J->n_mats; ++m) glass = glass || J->mats[m].type == 2;
    const int32_t g = (glass && J->max_depth > 0) ? 2 : 1;
    *pixels = pix;
    *rays = g == 2 ? (pix << J->max_depth) : pix;
    if (growth) *growth = g;
    return RG_OK;
}

constexpr int kEventRing = 32;

}  // namespace

// ------------------------------------------------------------ engine
struct rg_engine {
    rg_engine_desc d;
    hipStream_t st = nullptr;
    RgWaveBufs b;
    rg_pool pool;
    struct Frame {
        bool live = false;
        int64_t tag = 0, start = 0, last = 0, pix = 0;
        int32_t growth = 1;
        bool flags = false;              // its top level carries instance flags
        RgJobDev dev;
    };
    std::vector<Frame> frames;           // per slot
    int64_t pass = 0;                    // index of the next pass
    int64_t done_pass = 0;               // passes known complete
    hipEvent_t ev[kEventRing] = {};
    RgShadowSide side = {};              // shadow half of each pass on a second stream
    std::map<int64_t, std::vector<int32_t>> finishing;  // pass -> slots whose last pass it is
    std::vector<int64_t> done_tags;      // completed, not yet returned by poll
    int64_t admitted = 0, completed = 0, max_frames_in_pass = 0, max_depths_in_pass = 0;
};

namespace {

// Frees the host object and whatever HIP objects it holds (null ones skipped).
void engine_free(rg_engine *E) {
    for (int k = 0; k < kEventRing; ++k)
        if (E->ev[k]) (void)hipEventDestroy(E->ev[k]);
    if (E->side.shaded) (void)hipEventDestroy(E->side.shaded);
    if (E->side.shadowed) (void)hipEventDestroy(E->side.shadowed);
    if (E->side.st) (void)hipStreamDestroy(E->side.st);
    delete E;
}

// Moves passes that completed on the device into done_tags, releasing their
// frames.  block: wait for the oldest outstanding pass first.
rg_status harvest(rg_engine *E, bool block) {
    while (E->done_pass < E->pass) {
        hipEvent_t e = E->ev[E->done_pass % kEventRing];
        if (block) {
            RG_HIP(hipEventSynchronize(e));
            block = false;
        } else {
            hipError_t q = hipEventQuery(e);
            if (q == hipErrorNotReady) {
                (void)hipGetLastError();  // a pending pass is not an error for later checks
                break;
            }
            RG_HIP(q);
        }
        auto it = E->finishing.find(E->done_pass);
        if (it != E->finishing.end()) {
            for (int32_t s : it->second) {
                rg_engine::Frame &F = E->frames[(size_t)s];
                E->done_tags.push_back(F.tag);
                F.live = false;
                pool_release(E->pool, s);
                E->completed += 1;
            }
            E->finishing.erase(it);
        }
        E->done_pass += 1;
    }
    return RG_OK;
}

}  // namespace

extern "C" {

rg_status rg_pool_create(int64_t max_rays, int64_t max_pixels, int32_t max_jobs, rg_pool **out) {
    if (!out) return RG_ERR_INVALID_ARG;
    *out = nullptr;
    rg_pool *p = new (std::nothrow) rg_pool;
    if (!p) return RG_ERR_OUT_OF_MEMORY;
    if (!pool_init(*p, max_rays, max_pixels, max_jobs)) {
        delete p;
        return RG_ERR_INVALID_ARG;
    }
    *out = p;
    return RG_OK;
}

rg_status rg_pool_destroy(rg_pool *p) {
    delete p;
    return RG_OK;
}

rg_status rg_pool_reserve(rg_pool *p, int64_t rays, int64_t pixels, int32_t *slot, int64_t *pix_off) {
    if (!p || !slot || !pix_off) return RG_ERR_INVALID_ARG;
    return pool_reserve(*p, rays, pixels, slot, pix_off);
}

rg_status rg_pool_release(rg_pool *p, int32_t slot) {
    if (!p) return RG_ERR_INVALID_ARG;
    return pool_release(*p, slot);
}

rg_status rg_pool_get_usage(const rg_pool *p, rg_pool_usage *u) {
    if (!p || !u) return RG_ERR_INVALID_ARG;
    u->rays = p->rays_used;
    u->pixels = p->pixels_used;
    int64_t big = 0;
    for (const auto &kv : p->free_px) big = std::max(big, kv.second);
    u->largest_free_pixels = big;
    u->jobs = p->jobs_used;
    u->reserved = 0;
    return RG_OK;
}

rg_status rg_job_reservation(const rg_job *job, int64_t *rays, int64_t *pixels) {
    if (!rays || !pixels) return RG_ERR_INVALID_ARG;
    return reservation(job, rays, pixels, nullptr);
}

rg_status rg_engine_sizes(const rg_engine_desc *d, uint64_t *scratch_bytes) {
    if (!d || !scratch_bytes || d->max_rays < 1 || d->max_rays > (1ll << 31) || d->max_pixels < 1 ||
        d->max_pixels > (1ll << 31) || d->max_jobs < 1 || d->max_jobs > (1 << 20) || d->max_mats < 1 ||
        d->max_mats > 65536 || (int64_t)d->max_jobs * d->max_mats > (1ll << 31))
        return RG_ERR_INVALID_ARG;
    RgArena A{nullptr, 0, 0};
    RgWaveBufs b;
    rg_wave_carve(A, d->max_pixels, d->max_rays, d->max_jobs, (int64_t)d->max_jobs * d->max_mats, b);
    *scratch_bytes = A.used;
    return RG_OK;
}

rg_status rg_engine_create(const rg_engine_desc *d, void *scratch, uint64_t scratch_bytes, void *stream,
                           rg_engine **out) {
    if (!out) return RG_ERR_INVALID_ARG;
    *out = nullptr;
    uint64_t need = 0;
    rg_status r = rg_engine_sizes(d, &need);
    if (r != RG_OK) return r;
    if (!scratch || (d->width != 2 && d->width != 4 && d->width != 8)) return RG_ERR_INVALID_ARG;
    if (scratch_bytes < need) return RG_ERR_OUT_OF_MEMORY;
    rg_engine *E = new (std::nothrow) rg_engine;
    if (!E) return RG_ERR_OUT_OF_MEMORY;
    E->d = *d;
    E->st = (hipStream_t)stream;
    pool_init(E->pool, d->max_rays, d->max_pixels, d->max_jobs);
    E->frames.resize((size_t)d->max_jobs);
    RgArena A{(char *)scratch, scratch_bytes, 0};
    rg_wave_carve(A, d->max_pixels, d->max_rays, d->max_jobs, (int64_t)d->max_jobs * d->max_mats, E->b);
    hipError_t e = hipSuccess;
    for (int k = 0; k < kEventRing && e == hipSuccess; ++k)
        e = hipEventCreateWithFlags(&E->ev[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&E->side.shaded, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&E->side.shadowed, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&E->side.st, hipStreamNonBlocking);  // default priority
    if (e != hipSuccess) {
        engine_free(E);
        rg_set_error(__FILE__, __LINE__, hipGetErrorName(e));
        return RG_ERR_HIP;
    }
    r = rg_wave_reset(E->b, E->st);
    if (r != RG_OK) {
        engine_free(E);
        return r;
    }
    *out = E;
    return RG_OK;
}

rg_status rg_engine_destroy(rg_engine *E) {
    if (!E) return RG_OK;
    hipError_t e = hipStreamSynchronize(E->st);
    hipError_t e2 = E->side.st ? hipStreamSynchronize(E->side.st) : hipSuccess;
    if (e == hipSuccess) e = e2;
    engine_free(E);
    if (e != hipSuccess) {
        rg_set_error(__FILE__, __LINE__, hipGetErrorName(e));
        return RG_ERR_HIP;
    }
    return RG_OK;
}

rg_status rg_engine_admit(rg_engine *E, const rg_job *J, int64_t tag, int32_t *admitted) {
    if (!E || !J || !admitted) return RG_ERR_INVALID_ARG;
    *admitted = 0;
    const rg_tlas *t = J->tlas;
    if (!t || !t->buf || t->n_inst < 1 || !J->image) return RG_ERR_INVALID_ARG;
    if (J->mode != 0) return RG_ERR_UNSUPPORTED;
    if (t->width != E->d.width) return RG_ERR_UNSUPPORTED;
    if (!rg_trace_depth_ok(t)) return RG_ERR_UNSUPPORTED;
    if (J->n_mats > E->d.max_mats) return RG_ERR_INVALID_ARG;
    int64_t rays = 0, pix = 0;
    int32_t growth = 1;
    rg_status r = reservation(J, &rays, &pix, &growth);
    if (r != RG_OK) return r;
    int32_t slot = -1;
    int64_t off = -1;
    r = pool_reserve(E->pool, rays, pix, &slot, &off);
    if (r != RG_OK) return r;
    if (slot < 0) return RG_OK;  // no room now: the caller retries after a poll
    rg_engine::Frame &F = E->frames[(size_t)slot];
    RgJobDev &D = F.dev;
    D = RgJobDev{};
    D.cam = J->cam;
    D.light = J->light;
    D.pix_off = (uint32_t)off;
    D.width = (uint32_t)J->width;
    D.height = (uint32_t)J->height;
    D.mat_off = (uint32_t)((int64_t)slot * E->d.max_mats);
    D.n_mats = (uint32_t)J->n_mats;
    D.max_depth = J->max_depth;
    D.start = E->pass;
    D.image = J->image;
    RgTlasRef T = {(const char *)t->buf + t->nodes_off, (const RgInst *)((const char *)t->buf + t->inst_off)};
    r = rg_wave_put_job(E->b, (uint32_t)slot, D, T, J->mats, J->n_mats, E->st);
    if (r == RG_OK) r = rg_wave_camera(E->b, (uint32_t)slot, D, (int)(E->pass & 1), E->st);
    if (r != RG_OK) {
        pool_release(E->pool, slot);
        return r;
    }
    F.live = true;
    F.flags = t->has_inst_flags != 0;
    F.tag = tag;
    F.start = E->pass;
    F.last = E->pass + J->max_depth;
    F.pix = pix;
    F.growth = growth;
    E->finishing[F.last].push_back(slot);
    E->admitted += 1;
    *admitted = 1;
    return RG_OK;
}

rg_status rg_engine_step(rg_engine *E, int32_t *ran) {
    if (!E) return RG_ERR_INVALID_ARG;
    if (ran) *ran = 0;
    int64_t bound = 0, frames = 0;
    uint32_t depth_mask = 0;
    bool opt = false;
    for (const rg_engine::Frame &F : E->frames) {
        if (!F.live || F.last < E->pass) continue;
        const int64_t k = E->pass - F.start;
        bound += F.growth == 2 ? (F.pix << k) : F.pix;
        frames += 1;
        depth_mask |= 1u << k;
        opt = opt || F.flags;
    }
    if (frames == 0) return RG_OK;
    if (E->pass - E->done_pass >= kEventRing) {
        rg_status r = harvest(E, true);
        if (r != RG_OK) return r;
    }
    rg_status r = rg_wave_pass(E->b, E->d.width, E->pass, bound, E->st, RG_TUNE_ENGINE, opt, &E->side);
    if (r != RG_OK) return r;
    // the pass is complete once its shadow half (on the side stream) is
    auto it = E->finishing.find(E->pass);
    if (it != E->finishing.end())
        for (int32_t s : it->second) {
            r = rg_wave_resolve(E->b, E->frames[(size_t)s].dev, E->side.st);
            if (r != RG_OK) return r;
        }
    RG_HIP(hipEventRecord(E->ev[E->pass % kEventRing], E->side.st));
    E->pass += 1;
    E->max_frames_in_pass = std::max(E->max_frames_in_pass, frames);
    E->max_depths_in_pass = std::max<int64_t>(E->max_depths_in_pass, __builtin_popcount(depth_mask));
    if (ran) *ran = 1;
    return rg_debug_done(RG_OK, E->st);
}

rg_status rg_engine_poll(rg_engine *E, int32_t wait, int64_t *tags, int32_t cap, int32_t *n_done) {
    if (!E || !n_done || cap < 0 || (cap > 0 && !tags)) return RG_ERR_INVALID_ARG;
    *n_done = 0;
    rg_status r = harvest(E, wait != 0);
    if (r != RG_OK) return r;
    const int32_t n = (int32_t)std::min<size_t>((size_t)cap, E->done_tags.size());
    for (int32_t i = 0; i < n; ++i) tags[i] = E->done_tags[(size_t)i];
    E->done_tags.erase(E->done_tags.begin(), E->done_tags.begin() + n);
    *n_done = n;
    return RG_OK;
}

rg_status rg_engine_get_info(const rg_engine *E, rg_engine_info *out) {
    if (!E || !out) return RG_ERR_INVALID_ARG;
    int64_t live = 0, active = 0;
    for (const rg_engine::Frame &F : E->frames) {
        live += F.live;
        active += F.live && F.last >= E->pass;
    }
    out->passes = E->pass;
    out->passes_done = E->done_pass;
    out->frames_live = live;
    out->frames_active = active;
    out->admitted = E->admitted;
    out->completed = E->completed;
    out->rays_reserved = E->pool.rays_used;
    out->pixels_reserved = E->pool.pixels_used;
    out->max_frames_in_pass = E->max_frames_in_pass;
    out->max_depths_in_pass = E->max_depths_in_pass;
    return RG_OK;
}

rg_status rg_engine_stats(rg_engine *E, rg_render_stats *stats) {
    if (!E || !stats) return RG_ERR_INVALID_ARG;
    unsigned long long hs[2] = {0, 0};
    RG_HIP(hipStreamSynchronize(E->side.st));
    RG_HIP(hipMemcpyAsync(hs, E->b.stat, 16, hipMemcpyDeviceToHost, E->st));
    RG_HIP(hipStreamSynchronize(E->st));
    stats->rays_traced = hs[0];
    stats->shadow_rays = hs[1];
    stats->ms_total = 0.0f;
    return RG_OK;
}

}  // extern "C"
