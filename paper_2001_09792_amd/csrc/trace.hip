// trace.hip -- closest-hit / any-hit traversal kernels and their entry points
// (the per-ray closest hit, any hit and miss outcomes of the paper's
// section 1).  The traversal itself is in trace_core.h.
#include "trace_core.h"

namespace {

// Persistent traversal: each wave walks its own sequence of 64-ray packets
// (packets wave, wave + waves, wave + 2 waves, ... so that every wave samples
// the whole batch), and lanes whose ray has finished take the next rays of
// that sequence together, once at least `refill` lanes are idle.  Rays of a
// packet stay neighbours, and no lane idles while its wave has work left.
template <int W, bool ANY, int MODE, bool OPT>
__global__ void __launch_bounds__(rgt::kThreads) k_trace(RgTraceArgs a, int refill, int lds_depth, int leaf_batch,
                                                         int inst_batch) {
    extern __shared__ uint32_t lds_stack[];  // lds_depth * kThreads entries
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    // a device count never exceeds the launch size (the queue capacity)
    const int64_t n = a.count ? ((int64_t)*a.count < a.n ? (int64_t)*a.count : a.n) : a.n;
    const int64_t n_packets = (n + 63) >> 6;
    const int64_t wave = ((int64_t)blockIdx.x * rgt::kThreads + threadIdx.x) >> 6;
    const int64_t n_waves = (int64_t)gridDim.x * (rgt::kThreads / 64);
    rgt::Tracer<W, ANY, MODE, OPT> tr;
    tr.tlas_nodes = reinterpret_cast<const RgNode<W> *>(a.nodes);
    tr.recs = a.recs;
    uint32_t priv_stack[rgt::kPrivStack];
    tr.st.lds = (uint32_t RG_LDS *)&lds_stack[threadIdx.x];
    tr.st.priv = priv_stack;
    tr.st.n_lds = lds_depth;
    if (OPT) {
        tr.call_cull = a.ray_flags & (RG_RAY_CULL_BACK | RG_RAY_CULL_FRONT);
        tr.rmask = a.mask;
    }
    int64_t next = 0;  // position in this wave's ray sequence (the same in all lanes)
    int64_t ray_i = -1;
    bool has = false;
    // A finished ray's results stay in its lane until the lane takes its next
    // ray (or the wave ends): writing them then puts the stores next to the
    // new ray's loads, instead of making every round wait for stores.
    bool pend = false;
    auto write_result = [&]() {
        if (MODE == rgt::kCounts) {
            a.counts[3 * ray_i] = tr.h.n_nodes;
            a.counts[3 * ray_i + 1] = tr.h.n_tris;
            a.counts[3 * ray_i + 2] = tr.h.n_inst;
        } else {
            if (ANY && a.occluded) a.occluded[ray_i] = tr.found ? 1 : 0;
            if (a.t) a.t[ray_i] = tr.h.t;
            if (a.u) a.u[ray_i] = tr.h.u;
            if (a.v) a.v[ray_i] = tr.h.v;
            if (a.inst) a.inst[ray_i] = tr.h.inst;
            if (a.prim) a.prim[ray_i] = tr.h.prim;
        }
    };
    while (true) {
        // every ballot and every update of `next` below is executed by all
        // lanes together, so `next` stays uniform across the wave
        const uint64_t need = __ballot(!has);
        const int n_need = __popcll(need);
        if (n_need >= refill) {
            if (!has) {
                int64_t j = next + __popcll(need & lt);
                int64_t pkt = wave + (j >> 6) * n_waves;
                int64_t idx = pkt * 64 + (j & 63);
                if (pkt < n_packets && idx < n) {
                    if (pend) write_result();
                    rgt::Ray R;
                    R.o[0] = a.ray[0][idx]; R.o[1] = a.ray[1][idx]; R.o[2] = a.ray[2][idx];
                    R.d[0] = a.ray[3][idx]; R.d[1] = a.ray[4][idx]; R.d[2] = a.ray[5][idx];
                    R.tmin = a.ray[6][idx];
                    R.tmax = a.ray[7][idx];
                    ray_i = idx;
                    if (a.ray_job) {
                        const RgTlasRef J = a.jobs[a.ray_job[idx]];
                        tr.tlas_nodes = reinterpret_cast<const RgNode<W> *>(J.nodes);
                        tr.recs = J.recs;
                    }
                    has = tr.begin(R);
                    if (OPT) tr.rmask = a.ray_mask ? (uint32_t)a.ray_mask[idx] : a.mask;
                    pend = !has;  // empty interval: a miss without traversal
                }
            }
            next += n_need;
        }
        if (__ballot(has) == 0) {
            // no lane holds a ray after a refill attempt of all 64 lanes: the
            // sequence is exhausted once its next packet is past the end
            if (wave + (next >> 6) * n_waves >= n_packets) break;
            continue;
        }
        // Which kinds of unit run this round: inner nodes whenever a lane
        // has one; leaves and instance entries (each a long stretch of code
        // that runs for the whole wave if any lane needs it) once enough
        // lanes wait for one, or when nothing else is left.  A lane that
        // waits keeps its state; every round runs at least one kind present.
        const uint32_t my = has ? tr.kind() : 0u;
        const int n_inner = __popcll(__ballot(my == rgt::kUnitInner));
        const int n_leaf = __popcll(__ballot(my == rgt::kUnitLeaf));
        const int n_inst = __popcll(__ballot(my == rgt::kUnitInst));
        uint32_t run = n_inner ? rgt::kUnitInner : 0u;
        if (n_leaf && (n_leaf >= leaf_batch || n_inner == 0)) run |= rgt::kUnitLeaf;
        if (n_inst && (n_inst >= inst_batch || run == 0)) run |= rgt::kUnitInst;
        if ((run & my) != 0u && tr.step()) {  // my == 0 for lanes without a ray
            has = false;
            pend = true;
        }
    }
    if (pend) write_result();
}

// Launch parameters per family of calls (RG_TUNE_*): refill threshold,
// resident waves per CU, LDS stack entries per lane, lanes waiting at leaves
// / instance entries before a wave runs that code.  Incoherent ray batches
// gain from waiting lanes; the coherent rays of frames do not.
rg_trace_tune g_tune[RG_TUNE_SCOPES] = {
    {8, 16, 16, 12, 6},  // RG_TUNE_TRACE: rg_trace_closest / any / counts
    {8, 16, 16, 1, 1},   // RG_TUNE_FRAME: rg_render, rg_batch_render
    {8, 16, 16, 8, 1},   // RG_TUNE_ENGINE: rg_engine_step
};

}  // namespace

int rg_cu_count() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, c = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
            c = 256;
        cus = c;
    }
    return cus;
}

namespace {

unsigned persistent_blocks(int64_t n, int waves_per_cu) {
    int64_t want = (int64_t)rg_cu_count() * waves_per_cu / (rgt::kThreads / 64);
    int64_t need = rg_blocks(n, rgt::kThreads);
    return (unsigned)(need < want ? need : want);
}

template <int W, bool OPT>
void launch_mode(bool any, int mode, const RgTraceArgs &a, hipStream_t st, unsigned blocks, size_t shm,
                 const rg_trace_tune &t) {
    const int refill = t.refill, lds = t.lds_depth, lb = t.leaf_batch, ib = t.inst_batch;
    if (mode == rgt::kCounts) {
        if (any) k_trace<W, true, rgt::kCounts, OPT><<<blocks, rgt::kThreads, shm, st>>>(a, refill, lds, lb, ib);
        else k_trace<W, false, rgt::kCounts, OPT><<<blocks, rgt::kThreads, shm, st>>>(a, refill, lds, lb, ib);
    } else if (mode == rgt::kRender) {
        if (any) k_trace<W, true, rgt::kRender, OPT><<<blocks, rgt::kThreads, shm, st>>>(a, refill, lds, lb, ib);
        else k_trace<W, false, rgt::kRender, OPT><<<blocks, rgt::kThreads, shm, st>>>(a, refill, lds, lb, ib);
    } else {
        if (any) k_trace<W, true, rgt::kClosest, OPT><<<blocks, rgt::kThreads, shm, st>>>(a, refill, lds, lb, ib);
        else k_trace<W, false, rgt::kClosest, OPT><<<blocks, rgt::kThreads, shm, st>>>(a, refill, lds, lb, ib);
    }
}

template <int W>
rg_status launch_w(bool any, int mode, const RgTraceArgs &a, hipStream_t st, const rg_trace_tune &t) {
    unsigned blocks = persistent_blocks(a.n, t.waves_per_cu);
    size_t shm = (size_t)t.lds_depth * rgt::kThreads * sizeof(uint32_t);
    if (a.opt) launch_mode<W, true>(any, mode, a, st, blocks, shm, t);
    else launch_mode<W, false>(any, mode, a, st, blocks, shm, t);
    RG_LAUNCH_CHECK();
    return RG_OK;
}

bool rays_ok(const rg_rays &r) {
    return r.ox && r.oy && r.oz && r.dx && r.dy && r.dz && r.tmin && r.tmax;
}

void fill_rays(RgTraceArgs &a, const rg_rays &r) {
    a.ray[0] = r.ox; a.ray[1] = r.oy; a.ray[2] = r.oz;
    a.ray[3] = r.dx; a.ray[4] = r.dy; a.ray[5] = r.dz;
    a.ray[6] = r.tmin; a.ray[7] = r.tmax;
}

bool set_opts(RgTraceArgs &a, const rg_trace_opts *o) {
    if (!o) return true;
    if ((o->flags & ~(RG_RAY_CULL_BACK | RG_RAY_CULL_FRONT)) || o->mask > 0xFFu) return false;
    a.ray_flags = o->flags;
    a.mask = o->mask;
    a.ray_mask = o->ray_mask;
    a.opt = o->flags != 0u || o->mask != RG_INST_MASK_ALL || o->ray_mask != nullptr;
    return true;
}

bool tlas_ok(const rg_tlas *t) {
    return t && t->buf && t->n_inst >= 1 && (t->width == 2 || t->width == 4 || t->width == 8);
}

}  // namespace

bool rg_trace_depth_ok(const rg_tlas *t) {
    int64_t need = (int64_t)(t->width - 1) * (t->depth + t->max_blas_depth) + 1;
    return need <= rgt::kStackCap;
}

rg_status rg_trace_launch(int width, bool any, int mode, const RgTraceArgs &a, hipStream_t st, int scope) {
    if (a.n <= 0) return RG_OK;
    if (scope < 0 || scope >= RG_TUNE_SCOPES) return RG_ERR_INVALID_ARG;
    const rg_trace_tune t = g_tune[scope];
    if (width == 2) return rg_debug_done(launch_w<2>(any, mode, a, st, t), st);
    if (width == 4) return rg_debug_done(launch_w<4>(any, mode, a, st, t), st);
    if (width == 8) return rg_debug_done(launch_w<8>(any, mode, a, st, t), st);
    return RG_ERR_INVALID_ARG;
}

extern "C" {

rg_status rg_trace_tuning(int32_t scope, const rg_trace_tune *set, rg_trace_tune *get) {
    if (scope < 0 || scope >= RG_TUNE_SCOPES) return RG_ERR_INVALID_ARG;
    if (set) {
        if (set->refill < 1 || set->refill > 64 || set->waves_per_cu < 4 || set->waves_per_cu > 64 ||
            set->lds_depth < 8 || set->lds_depth > rgt::kMaxLdsStack || set->leaf_batch < 1 ||
            set->leaf_batch > 64 || set->inst_batch < 1 || set->inst_batch > 64)
            return RG_ERR_INVALID_ARG;
        g_tune[scope] = *set;
    }
    if (get) *get = g_tune[scope];
    return RG_OK;
}

rg_status rg_trace_closest(const rg_tlas *tlas, rg_rays rays, int64_t n, rg_hits out, void *stream) {
    return rg_trace_closest_ex(tlas, rays, n, out, nullptr, stream);
}

rg_status rg_trace_any(const rg_tlas *tlas, rg_rays rays, int64_t n, uint8_t *occluded, const rg_hits *found,
                       void *stream) {
    return rg_trace_any_ex(tlas, rays, n, occluded, found, nullptr, stream);
}

rg_status rg_trace_closest_ex(const rg_tlas *tlas, rg_rays rays, int64_t n, rg_hits out, const rg_trace_opts *opts,
                              void *stream) {
    if (!tlas_ok(tlas) || n < 0 || (n > 0 && !rays_ok(rays))) return RG_ERR_INVALID_ARG;
    RgTraceArgs a = {};
    if (!set_opts(a, opts)) return RG_ERR_INVALID_ARG;
    a.opt = a.opt || tlas->has_inst_flags != 0;
    if (!rg_trace_depth_ok(tlas)) return RG_ERR_UNSUPPORTED;
    if (n == 0) return RG_OK;
    a.nodes = (const char *)tlas->buf + tlas->nodes_off;
    a.recs = (const RgInst *)((const char *)tlas->buf + tlas->inst_off);
    fill_rays(a, rays);
    a.n = n;
    a.t = out.t; a.u = out.u; a.v = out.v; a.inst = out.inst; a.prim = out.prim;
    return rg_trace_launch(tlas->width, false, rgt::kClosest, a, (hipStream_t)stream, RG_TUNE_TRACE);
}

rg_status rg_trace_any_ex(const rg_tlas *tlas, rg_rays rays, int64_t n, uint8_t *occluded, const rg_hits *found,
                          const rg_trace_opts *opts, void *stream) {
    if (!tlas_ok(tlas) || n < 0 || (n > 0 && (!rays_ok(rays) || !occluded))) return RG_ERR_INVALID_ARG;
    RgTraceArgs a = {};
    if (!set_opts(a, opts)) return RG_ERR_INVALID_ARG;
    a.opt = a.opt || tlas->has_inst_flags != 0;
    if (!rg_trace_depth_ok(tlas)) return RG_ERR_UNSUPPORTED;
    if (n == 0) return RG_OK;
    a.nodes = (const char *)tlas->buf + tlas->nodes_off;
    a.recs = (const RgInst *)((const char *)tlas->buf + tlas->inst_off);
    fill_rays(a, rays);
    a.n = n;
    a.occluded = occluded;
    if (found) {
        a.t = found->t; a.u = found->u; a.v = found->v; a.inst = found->inst; a.prim = found->prim;
    }
    return rg_trace_launch(tlas->width, true, rgt::kClosest, a, (hipStream_t)stream, RG_TUNE_TRACE);
}

rg_status rg_trace_counts(const rg_tlas *tlas, rg_rays rays, int64_t n, int32_t any_hit, uint32_t *counts,
                          void *stream) {
    if (!tlas_ok(tlas) || n < 0 || (n > 0 && (!rays_ok(rays) || !counts))) return RG_ERR_INVALID_ARG;
    if (!rg_trace_depth_ok(tlas)) return RG_ERR_UNSUPPORTED;
    if (n == 0) return RG_OK;
    RgTraceArgs a = {};
    a.nodes = (const char *)tlas->buf + tlas->nodes_off;
    a.recs = (const RgInst *)((const char *)tlas->buf + tlas->inst_off);
    fill_rays(a, rays);
    a.n = n;
    a.counts = counts;
    a.opt = tlas->has_inst_flags != 0;
    return rg_trace_launch(tlas->width, any_hit != 0, rgt::kCounts, a, (hipStream_t)stream, RG_TUNE_TRACE);
}

}  // extern "C"
