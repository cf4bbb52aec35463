// trace.hip -- closest-hit / any-hit traversal kernels and their entry points
// (the per-ray closest hit, any hit and miss outcomes of the paper's
// section 1).  The traversal itself is in trace_core.h.
#include "trace_core.h"

namespace {

template <int W, bool ANY, int MODE>
__global__ void __launch_bounds__(rgt::kThreads) k_trace(RgTraceArgs a) {
    __shared__ uint32_t lds_stack[rgt::kLdsStack * rgt::kThreads];
    int64_t i = blockIdx.x * (int64_t)rgt::kThreads + threadIdx.x;
    int64_t n = a.count ? (int64_t)*a.count : a.n;
    if (i >= n) return;
    rgt::Ray R;
    R.o[0] = a.ray[0][i]; R.o[1] = a.ray[1][i]; R.o[2] = a.ray[2][i];
    R.d[0] = a.ray[3][i]; R.d[1] = a.ray[4][i]; R.d[2] = a.ray[5][i];
    R.tmin = a.ray[6][i];
    R.tmax = a.ray[7][i];
    rgt::Hit h;
    bool f = rgt::trace_ray<W, ANY, MODE>(reinterpret_cast<const RgNode<W> *>(a.nodes), a.recs, R,
                                          &lds_stack[threadIdx.x], h);
    if (MODE == rgt::kCounts) {
        a.counts[3 * i] = h.n_nodes;
        a.counts[3 * i + 1] = h.n_tris;
        a.counts[3 * i + 2] = h.n_inst;
        return;
    }
    if (ANY && a.occluded) a.occluded[i] = f ? 1 : 0;
    if (a.t) a.t[i] = h.t;
    if (a.u) a.u[i] = h.u;
    if (a.v) a.v[i] = h.v;
    if (a.inst) a.inst[i] = h.inst;
    if (a.prim) a.prim[i] = h.prim;
}

template <int W>
rg_status launch_w(bool any, int mode, const RgTraceArgs &a, hipStream_t st) {
    unsigned blocks = rg_blocks(a.n, rgt::kThreads);
    if (mode == rgt::kCounts) {
        if (any) k_trace<W, true, rgt::kCounts><<<blocks, rgt::kThreads, 0, st>>>(a);
        else k_trace<W, false, rgt::kCounts><<<blocks, rgt::kThreads, 0, st>>>(a);
    } else if (mode == rgt::kRender) {
        if (any) k_trace<W, true, rgt::kRender><<<blocks, rgt::kThreads, 0, st>>>(a);
        else k_trace<W, false, rgt::kRender><<<blocks, rgt::kThreads, 0, st>>>(a);
    } else {
        if (any) k_trace<W, true, rgt::kClosest><<<blocks, rgt::kThreads, 0, st>>>(a);
        else k_trace<W, false, rgt::kClosest><<<blocks, rgt::kThreads, 0, st>>>(a);
    }
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

bool tlas_ok(const rg_tlas *t) {
    return t && t->buf && t->n_inst >= 1 && (t->width == 2 || t->width == 4 || t->width == 8);
}

}  // namespace

bool rg_trace_depth_ok(const rg_tlas *t) {
    int64_t need = (int64_t)(t->width - 1) * (t->depth + t->max_blas_depth) + 1;
    return need <= rgt::kStackCap;
}

rg_status rg_trace_launch(int width, bool any, int mode, const RgTraceArgs &a, hipStream_t st) {
    if (a.n <= 0) return RG_OK;
    if (width == 2) return launch_w<2>(any, mode, a, st);
    if (width == 4) return launch_w<4>(any, mode, a, st);
    if (width == 8) return launch_w<8>(any, mode, a, st);
    return RG_ERR_INVALID_ARG;
}

extern "C" {

rg_status rg_trace_closest(const rg_tlas *tlas, rg_rays rays, int64_t n, rg_hits out, void *stream) {
    if (!tlas_ok(tlas) || n < 0 || (n > 0 && !rays_ok(rays))) return RG_ERR_INVALID_ARG;
    if (!rg_trace_depth_ok(tlas)) return RG_ERR_UNSUPPORTED;
    if (n == 0) return RG_OK;
    RgTraceArgs a = {};
    a.nodes = (const char *)tlas->buf + tlas->nodes_off;
    a.recs = (const RgInst *)((const char *)tlas->buf + tlas->inst_off);
    fill_rays(a, rays);
    a.n = n;
    a.t = out.t; a.u = out.u; a.v = out.v; a.inst = out.inst; a.prim = out.prim;
    return rg_trace_launch(tlas->width, false, rgt::kClosest, a, (hipStream_t)stream);
}

rg_status rg_trace_any(const rg_tlas *tlas, rg_rays rays, int64_t n, uint8_t *occluded, const rg_hits *found,
                       void *stream) {
    if (!tlas_ok(tlas) || n < 0 || (n > 0 && (!rays_ok(rays) || !occluded))) return RG_ERR_INVALID_ARG;
    if (!rg_trace_depth_ok(tlas)) return RG_ERR_UNSUPPORTED;
    if (n == 0) return RG_OK;
    RgTraceArgs a = {};
    a.nodes = (const char *)tlas->buf + tlas->nodes_off;
    a.recs = (const RgInst *)((const char *)tlas->buf + tlas->inst_off);
    fill_rays(a, rays);
    a.n = n;
    a.occluded = occluded;
    if (found) {
        a.t = found->t; a.u = found->u; a.v = found->v; a.inst = found->inst; a.prim = found->prim;
    }
    return rg_trace_launch(tlas->width, true, rgt::kClosest, a, (hipStream_t)stream);
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
    return rg_trace_launch(tlas->width, any_hit != 0, rgt::kCounts, a, (hipStream_t)stream);
}

}  // extern "C"
