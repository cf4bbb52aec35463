// wavefront.h -- buffers and passes of the breadth-first Whitted loop,
// shared by the per-frame / batched renderer (render.hip) and the serving
// engine (serve.hip).
//
// A pass traces every queued ray of every frame at once (closest hit),
// shades the hits (sky, ambient, shadow rays, mirror and glass children),
// traces the shadow rays (any hit) and adds the direct term of the
// unoccluded ones.  A queue entry carries its frame (job slot); the frame's
// record gives its camera, light, materials, accumulator range and the pass
// at which its camera rays were traced (`start`), so frames at different
// recursion depths share one pass.
#pragma once

#include "trace_core.h"

// A queue entry is a ray plus its payload: the pixel (index into the
// accumulators), the frame (job slot) it belongs to and its throughput.
struct RgQueue {
    float *ray[8];
    uint32_t *pix, *job;
    float *beta[3];
};
struct RgShadowQ {
    float *ray[8];
    uint32_t *pix, *job;
    float *pend[3];
    uint8_t *occ;
};

// One frame as the kernels see it.  Depth of an entry = pass - start.
struct RgJobDev {
    rg_camera cam;
    rg_light light;
    uint32_t pix_off, width, height, mat_off, n_mats;
    int32_t max_depth;
    int64_t start;
    float *image;
    uint32_t *gbuf;  // nullable: the material each primary ray shaded (RG_MISS: sky)
};

// Device buffers of a wavefront render, carved from one caller buffer:
// accumulators (3 x u64 per pixel), statistics, queue counters (0, 1: the
// two ray queues, 2: the shadow queue), frame / top-level / material tables,
// hit arrays, two ray queues and a shadow queue of `cap` entries each.
struct RgWaveBufs {
    unsigned long long *acc, *stat;
    uint32_t *counts;
    RgJobDev *jobs;
    RgTlasRef *tlas;
    RgMat *mats;
    float *hit_t;
    uint32_t *hit_rec, *hit_slot;
    RgQueue q[2];
    RgShadowQ sq;
    int64_t cap;
};

// Carves the buffers (base NULL: sizing pass, A.used = bytes).  False when
// the arena is too small.
bool rg_wave_carve(RgArena &A, int64_t pixels, int64_t cap, int64_t n_jobs, int64_t n_mats, RgWaveBufs &b);

// Zeroes the statistics and the three queue counters.
rg_status rg_wave_reset(const RgWaveBufs &b, hipStream_t st);

// Writes frame record `slot` (and its top-level reference) and n_mats
// materials at b.mats + J.mat_off, through kernel arguments, so the host
// arrays may go away when this returns and nothing waits; zeroes the
// frame's accumulators.
rg_status rg_wave_put_job(const RgWaveBufs &b, uint32_t slot, const RgJobDev &J, const RgTlasRef &T,
                          const rg_material *host_mats, int32_t n_mats, hipStream_t st);

// Appends the frame's camera rays (one per pixel) to ray queue `queue`.
rg_status rg_wave_camera(const RgWaveBufs &b, uint32_t slot, const RgJobDev &J, int queue, hipStream_t st);

// A second stream for the shadow half of each pass.  The shadow rays of
// pass p are traced and their direct term added on `st` while the main
// stream runs the closest-hit traversal of pass p+1 (the persistent kernels
// of one fill the tail of the other).  `shaded` orders the shadow work after
// the shading that queued it; `shadowed` orders the next pass's reuse of the
// shadow queue after it.  Events owned by the caller.
struct RgShadowSide {
    hipStream_t st;
    hipEvent_t shaded, shadowed;
    bool pending;  // shadow work of an earlier pass was enqueued on st
};

// One pass over ray queue (pass & 1): closest hit, shading into the other
// ray queue, shadow any hit, direct term.  `bound` >= the entries queued
// (sizes the launches); width = node width of every top level involved.
// With `side`, the shadow half runs on side->st (see above): work that needs
// the pass complete (image resolves) goes to side->st as well.
// scope: the RG_TUNE_* launch parameters of the traversals; opt: some
// frame's top level carries instance flags (masks, cull flags).
rg_status rg_wave_pass(const RgWaveBufs &b, int32_t width, int64_t pass, int64_t bound, hipStream_t st,
                       int scope, bool opt, RgShadowSide *side = nullptr);

// Converts the frame's accumulators to its float RGB image.
rg_status rg_wave_resolve(const RgWaveBufs &b, const RgJobDev &J, hipStream_t st);
