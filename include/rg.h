/*
 * rg.h -- C ABI of the MI355X ray-tracing library (librg.so).
 *
 * The paper describes ray tracing on RTX as two steps (section 1): first a
 * two-layered structure is built from the vertex data of the scene's models
 * and their transformation matrices; then a dispatch runs a ray-generation
 * shader, and for each ray a closest-hit, any-hit or miss shader runs, which
 * may spawn further rays up to a recursion limit (footnote), each ray carrying
 * a small payload.  Section 2.1 adds multiple objects, reflection, refraction
 * and shadow casting.  This header turns those steps into calls:
 *
 *   bottom level from vertex data            rg_build_blas   (+ rg_blas_sizes;
 *                                            enqueued: rg_build_blas_async /
 *                                            rg_build_blas_finish)
 *   top level from instances and matrices    rg_build_tlas   (+ rg_tlas_sizes;
 *                                            enqueued: rg_build_tlas_async /
 *                                            rg_build_tlas_finish)
 *   ray generation                           rg_camera_rays, rg_ao_rays
 *   closest hit / miss per ray               rg_trace_closest
 *   any hit per ray                          rg_trace_any
 *   dispatch with capped recursion/payload   rg_render       (+ rg_render_sizes)
 *
 * Conventions (all entry points):
 *   - Pointers are DEVICE pointers unless the comment says "host".
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it; calls documented as "synchronous" also wait for
 *     it before returning.
 *   - The library never allocates device memory: the caller allocates every
 *     buffer, sized with the *_sizes calls.  Buffers must be 256-byte aligned
 *     (any torch CUDA tensor's storage is).
 *   - Return value: RG_OK or a negative rg_status.  Argument validation is
 *     done on the host before anything is enqueued; a failed validation
 *     enqueues nothing.  Device faults surface at the caller's next sync.
 *   - Nothing throws across the ABI.  The library is thread-safe for calls on
 *     different buffers; concurrent calls that share a scratch buffer race.
 *
 * Ray semantics: a ray is o + t d with t in the closed interval [tmin, tmax];
 * t is measured in units of |d| (directions need not be unit length).
 * Triangles are two-sided, their edges and vertices count as inside, and a
 * ray parallel to a triangle's plane misses it.  Closest hit returns the least
 * t; exact ties go to the lowest (instance, primitive).  Barycentrics follow
 * p = (1-u-v) v0 + u v1 + v v2.  A miss is reported as t = +inf and
 * inst = prim = RG_MISS.
 */
#ifndef RG_H
#define RG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rg_status;
#define RG_OK 0
#define RG_ERR_INVALID_ARG (-1)   /* bad pointer, size, value or option */
#define RG_ERR_OUT_OF_MEMORY (-2) /* a caller buffer is smaller than *_sizes reported */
#define RG_ERR_HIP (-3)           /* a HIP runtime call or kernel launch failed */
#define RG_ERR_UNSUPPORTED (-4)   /* valid request outside what this build handles */
#define RG_ERR_UNIMPLEMENTED (-5)
/* Asynchronous calls (tracing, rendering, batches, the engine's step, refits,
 * opacity masks, post-process passes, ray generation) only enqueue work: a
 * device fault surfaces at the caller's next synchronisation.  With RG_DEBUG=1
 * in the environment (read once per process) each of them waits for its
 * stream before returning and reports a failed launch or a fault as
 * RG_ERR_HIP (rg_last_error() names it). */

#define RG_MISS 0xFFFFFFFFu
#define RG_PER_PRIM 0xFFFFFFFFu   /* instance material: use the mesh's per-primitive ids */
#define RG_MAX_DEPTH 8
#define RG_LEVELS_CAP 255        /* deepest bottom level whose level table is kept */

/* Hierarchy builders.  Both start from the primitives sorted by the Morton
 * code of their box centres.
 *   RG_BUILDER_LBVH: Karras's radix tree over the sorted codes, boxes refit
 *     bottom-up (the linear BVH the paper's GPU build follows).
 *   RG_BUILDER_PLOC: parallel locally-ordered clustering (Meister & Bittner
 *     2018): each round every cluster takes the neighbour, within `radius`
 *     positions of the sorted cluster list, whose union box has the least
 *     surface area (float32; ties to the nearer-to-front position); mutual
 *     nearest pairs merge into the lower position; repeated down to one
 *     cluster.  Slower to build, tighter boxes, fewer node visits.
 *   RG_BUILDER_TREELET: the linear BVH, then rounds of treelet
 *     restructuring (Karras & Aila 2013): at every inner node with at least
 *     three leaves below it (each after the nodes below it), a treelet of up
 *     to 7 leaves grown by repeatedly opening its inner leaf of largest
 *     surface area is rebuilt with the topology of least total float32
 *     surface area (dynamic programming over the leaf subsets); the leaves
 *     are then renumbered in the tree's left-to-right order. */
#define RG_BUILDER_LBVH 0
#define RG_BUILDER_PLOC 1
#define RG_BUILDER_TREELET 2
#define RG_PLOC_RADIUS_DEFAULT 16
#define RG_TREELET_ROUNDS_DEFAULT 3

/* Hierarchy options.  width = children per node (2, 4 or 8); leaf_max =
 * most triangles per leaf (1..8); builder = RG_BUILDER_*; radius = search
 * radius of RG_BUILDER_PLOC (1..32, 0 = RG_PLOC_RADIUS_DEFAULT), rounds of
 * RG_BUILDER_TREELET (1..8, 0 = RG_TREELET_ROUNDS_DEFAULT), ignored by
 * RG_BUILDER_LBVH; morton_bits = bits per axis of the Morton codes: 21 (0
 * means 21: 63-bit keys, eight radix-sort passes) or 10 (30-bit keys, four
 * passes, for builds of at most 2^20 primitives: the key is the 21-bit key's
 * top 30 bits, a coarser grid that costs some hierarchy quality).  NULL
 * means {4, 4, RG_BUILDER_LBVH, 0, 0}. */
#define RG_MORTON_BITS_COMPACT_MAX_PRIMS (1 << 20)
typedef struct {
    int32_t width;
    int32_t leaf_max;
    int32_t builder;
    int32_t radius;
    int32_t morton_bits;
} rg_build_opts;

typedef struct {
    uint64_t bytes;         /* size of the output buffer */
    uint64_t scratch_bytes; /* size of the scratch buffer */
} rg_sizes;

/* Bottom-level structure: a POD descriptor of the caller's output buffer.
 * Layout of `buf` (all offsets in bytes from buf):
 *   0:         128-byte header: four uint64 device addresses (nodes, tris,
 *              mats, slots: the arrays below), the root box float lo[3],
 *              hi[3] (kept current by rg_refit_blas), uint32 status of the
 *              last refit's input check (0: valid), uint32 padding, uint64
 *              device address of the opacity masks (0: none), uint32 their
 *              level, padding.
 *   nodes_off: n_nodes nodes of 32*width bytes (width 4: 128 B):
 *              float lo_x[w], lo_y[w], lo_z[w], hi_x[w], hi_y[w], hi_z[w];
 *              uint32 child[w]; padding to 32*width bytes.
 *              child = RG_MISS: empty slot (its box is lo=+inf, hi=-inf);
 *              bit 31 clear: index of an inner node; bit 31 set: a leaf of
 *              bits 28..30 + 1 primitives starting at bits 0..27.
 *              Node 0 is the root.
 *   tris_off:  n_tris triangles in leaf order, 40 B each:
 *              float v0[3], v1[3], v2[3]; uint32 prim (index in the input).
 *   mats_off:  uint16 material per triangle in leaf order (0 if none given).
 *   slots_off: uint32 per input triangle: its position in leaf order.
 *   parents_off: uint32 per node: (parent node << 3) | the parent's child
 *              slot holding it; RG_MISS for the root (used by rg_refit_blas).
 *   levels_off: uint32[RG_LEVELS_CAP + 1]: nodes are numbered level by level
 *              (root level 0); entry l is the first node of level l and entry
 *              `depth` the node count (written when depth <= RG_LEVELS_CAP).
 * The build reads the vertex and index arrays only during the call; the
 * descriptor refers to `buf`, which must outlive every top level using it. */
typedef struct {
    void *buf;
    uint64_t nodes_off, tris_off, mats_off, slots_off, parents_off, levels_off;
    int64_t n_tris, n_nodes;
    int32_t width, leaf_max, depth, has_mats;
    float lo[3], hi[3]; /* root box (object space) at build time; the header holds the current one */
    int32_t has_alpha, alpha_level; /* opacity masks attached by rg_blas_set_alpha */
} rg_blas;

/* Top-level structure.  Layout of `buf`:
 *   nodes_off: nodes as above; leaves hold one instance each.
 *   inst_off:  n_inst 112-byte records in leaf order:
 *              float inv[9] (world->object linear part, row-major),
 *              float p[3] (object->world translation),
 *              uint64 blas_nodes, blas_tris, blas_header (device addresses),
 *              uint32 material (RG_PER_PRIM = per primitive), uint32 inst
 *              (index in the input), float blas_lo[3], blas_hi[3] (the
 *              bottom level's root box), 8 bytes of padding.
 *   rec_off:   uint32 per input instance: its record's position.
 *   xf_off:    float[n_inst][3][4]: the object->world matrices as given,
 *              in input order (the trace calls recompute reported hits
 *              from them).
 * It refers to the bottom levels' buffers, which must outlive it. */
typedef struct {
    void *buf;
    uint64_t nodes_off, inst_off, rec_off, xf_off;
    int64_t n_inst, n_nodes;
    int32_t width, depth, max_blas_depth;
    int32_t has_inst_flags; /* 1 when some instance carries flags other than RG_INST_MASK_ALL */
    float lo[3], hi[3]; /* world box */
} rg_tlas;

/* Rays in structure-of-arrays form, n entries each (device). */
typedef struct {
    const float *ox, *oy, *oz, *dx, *dy, *dz, *tmin, *tmax;
} rg_rays;

/* Hit records in structure-of-arrays form (device).  Any pointer may be
 * NULL to skip that field, except that t, u and v are computed from the hit's
 * identity: a call that asks for any of them must also pass inst and prim.
 * Miss: t = +inf, inst = prim = RG_MISS, u = v = 0. */
typedef struct {
    float *t;
    uint32_t *inst, *prim;
    float *u, *v;
} rg_hits;

typedef struct {
    int32_t type; /* 0 diffuse, 1 mirror, 2 glass */
    float rgb[3]; /* diffuse albedo or mirror reflectance; unused by glass */
    float ior;    /* glass index of refraction */
} rg_material;

typedef struct {
    float eye[3], target[3], up[3], vfov_deg; /* vertical field of view */
} rg_camera;

typedef struct {
    float pos[3], intensity[3], ambient;
} rg_light;

typedef struct {
    uint64_t rays_traced;  /* closest-hit rays of all depths */
    uint64_t shadow_rays;  /* any-hit rays (shadow or occlusion) */
    float ms_total;        /* GPU time of the whole call */
} rg_render_stats;

/* ---------------------------------------------------------------- errors */
const char *rg_status_string(rg_status s);
/* The last HIP failure of the calling thread as "file:line: hipErrorName"
 * (empty if none).  The pointer stays valid until the thread's next call. */
const char *rg_last_error(void);

/* ------------------------------------------------------- bottom level */
/* Sizes for a bottom level of n_tris triangles (host call, no GPU work).
 * Errors: RG_ERR_INVALID_ARG for n_tris < 1 or > 2^28, bad opts (also
 * morton_bits 10 with more than 2^20 triangles), NULL out. */
rg_status rg_blas_sizes(int64_t n_tris, const rg_build_opts *opts, rg_sizes *out /*host*/);

/* The bottom level of the two-level structure, built from a mesh's vertex
 * data (section 1: the first of the two steps, an acceleration structure per
 * mesh).  Builds a binary BVH (Morton codes of triangle-box centres, LSD
 * radix sort with LDS ranking, then opts' builder: Karras's radix tree with
 * inner boxes from the leaf ranges, locally-ordered clustering, or the radix
 * tree restructured by treelets) and collapses it into `width`-wide nodes
 * with leaves of at most leaf_max triangles; writes a header, nodes,
 * triangles in leaf order, per-triangle materials, per-node parents and the
 * level table into out_buf (offsets in *out).  verts: device
 * float[n_verts][3]; idx: device uint32[n_tris][3]; prim_material: device
 * uint16[n_tris] or NULL.  out_buf (rg_blas_sizes bytes) belongs to the
 * caller and must outlive every top level, trace and render over it;
 * scratch (rg_blas_sizes' scratch_bytes) is free again when the call
 * returns.  Synchronous (returns after `stream` has finished the build);
 * meshes of up to 4,096 triangles build in one workgroup.
 * Errors: RG_ERR_INVALID_ARG for NULL pointers, sizes out of range, an index
 * >= n_verts or a non-finite vertex (checked on the device: the clustering
 * and treelet builders wait for the check before building; the linear build
 * runs on the clamped input and reports it at its one final wait, leaving
 * out_buf unusable); RG_ERR_OUT_OF_MEMORY if out_bytes / scratch_bytes are
 * too small. */
rg_status rg_build_blas(const float *verts, int64_t n_verts, const uint32_t *idx, int64_t n_tris,
                        const uint16_t *prim_material, const rg_build_opts *opts,
                        void *out_buf, uint64_t out_bytes, void *scratch, uint64_t scratch_bytes,
                        void *stream, rg_blas *out /*host*/);

/* rg_build_blas without the wait (section 1's first step, enqueued): the
 * whole build of the linear builder (RG_BUILDER_LBVH; others:
 * RG_ERR_UNSUPPORTED) goes onto `stream` and the call returns; the
 * descriptor comes from rg_build_blas_finish.  ticket: RG_BUILD_TICKET_BYTES
 * of pinned host memory (hipHostMalloc or a pinned tensor), 16-byte
 * aligned, owned by the caller: the build's summary lands there by
 * asynchronous copies.  verts, idx, prim_material, out_buf, scratch and the
 * ticket must stay untouched until rg_build_blas_finish returns (so builds
 * that overlap need scratch buffers of their own).  Arguments, sizes and
 * errors detected on the host as rg_build_blas, returned at once. */
#define RG_BUILD_TICKET_BYTES 1024
rg_status rg_build_blas_async(const float *verts, int64_t n_verts, const uint32_t *idx, int64_t n_tris,
                              const uint16_t *prim_material, const rg_build_opts *opts, void *out_buf,
                              uint64_t out_bytes, void *scratch, uint64_t scratch_bytes, void *stream,
                              void *ticket /*pinned host*/);

/* Completes an rg_build_blas_async: waits until its stream has finished that
 * build (not the work queued after it), fills *out (as rg_build_blas does)
 * and returns the build's error: RG_ERR_INVALID_ARG for an index >= n_verts
 * or a non-finite vertex (found on the device), or for a ticket that holds
 * no pending build (each completes once).  A hierarchy deeper than the
 * levels the asynchronous call launched (rare: more than about 1.6 log_W
 * n_tris + 2) gets its remaining levels here, on the build's stream, with a
 * wait for them. */
rg_status rg_build_blas_finish(void *ticket /*pinned host*/, rg_blas *out /*host*/);

/* Scratch for rg_refit_blas on `blas` (host call, no GPU work). */
rg_status rg_refit_sizes(const rg_blas *blas /*host*/, uint64_t *scratch_bytes /*host*/);

/* Refits a bottom level built by rg_build_blas to new positions of the same
 * triangles (dynamic scenes: the per-frame update of moving geometry, the
 * step before tracing that the paper's scene graph and physics drive): idx
 * must be the index array of the build (n_tris equal), verts the new
 * float[n_verts][3].  The triangles in leaf order are rewritten and every
 * node box is recomputed bottom-up, one launch per level (min / max, exact:
 * unchanged vertices reproduce the build bit for bit); the hierarchy itself
 * is kept, so its quality degrades as triangles move far from where they were
 * built.  The new root box goes to the buffer's header, not to *blas.
 * Top levels over this bottom level carry its root box and must be rebuilt
 * (rg_build_tlas reads the root boxes from the headers) before tracing.
 * scratch: rg_refit_sizes bytes, used only by hierarchies deeper than
 * RG_LEVELS_CAP levels (may be NULL otherwise).  Asynchronous.
 * Errors: RG_ERR_INVALID_ARG for NULL pointers or another n_tris;
 * RG_ERR_OUT_OF_MEMORY for a short scratch buffer.  An index >= n_verts or a
 * non-finite vertex is found on the device: it sets the header's status word
 * (the offending triangles keep their old data, nothing is read out of
 * bounds), rg_build_tlas over this bottom level then fails with
 * RG_ERR_INVALID_ARG, and a later valid refit clears it. */
rg_status rg_refit_blas(rg_blas *blas /*host*/, const float *verts, int64_t n_verts,
                        const uint32_t *idx, int64_t n_tris, void *scratch, uint64_t scratch_bytes,
                        void *stream);

/* rg_refit_blas for n_blas bottom levels of one width at once (arrays of
 * n_blas host entries: descriptors, device pointers to each one's new
 * vertices and its index array, vertex and triangle counts): each launch
 * covers one level of all of them, so a set of meshes costs about what the
 * largest one costs.  scratch: the largest rg_refit_sizes among those deeper
 * than RG_LEVELS_CAP (NULL if none is).  Asynchronous.  Errors as
 * rg_refit_blas, and RG_ERR_INVALID_ARG for mixed widths. */
rg_status rg_refit_blas_many(rg_blas *blas /*host [n_blas]*/, int32_t n_blas,
                             const float *const *verts /*host [n_blas]*/, const int64_t *n_verts /*host*/,
                             const uint32_t *const *idx /*host [n_blas]*/, const int64_t *n_tris /*host*/,
                             void *scratch, uint64_t scratch_bytes, void *stream);

/* Opacity masks: the accept / ignore decision an any-hit stage takes for
 * alpha-tested geometry, per point of a triangle.  Each triangle is cut into
 * 4^level micro-triangles by splitting every edge into n = 2^level equal
 * parts; with (u, v) the barycentric weights of its second and third vertex
 * (those of rg_hits), scaled by n, the cell (i, j) = (floor(n u), floor(n v))
 * holds an upright micro-triangle (fractional parts summing to at most 1)
 * and, unless it touches the far edge, an inverted one; they are numbered
 * row by row, row j starting at j (2n - j), upright 2i, inverted 2i + 1.  Bit
 * k of a triangle's mask set: hits on micro-triangle k are accepted, else the
 * ray passes through.  alpha: device uint64[n_tris] in input order, read
 * while tracing (it must outlive every trace and render of the bottom level),
 * NULL to remove the masks; level 0..RG_ALPHA_LEVEL_MAX.  Writes the buffer's
 * header (asynchronous, on `stream`) and updates *blas; top levels over the
 * bottom level must be built again afterwards.  The masks apply to every
 * trace and render call.  Errors: RG_ERR_INVALID_ARG. */
#define RG_ALPHA_LEVEL_MAX 3
rg_status rg_blas_set_alpha(rg_blas *blas, const uint64_t *alpha, int32_t level, void *stream);

/* Reads a bottom level's header: current root box and the status of its last
 * refit (0: valid input).  Synchronous (waits for `stream`). */
rg_status rg_blas_state(const rg_blas *blas /*host*/, float *lo /*host [3]*/, float *hi /*host [3]*/,
                        uint32_t *status /*host*/, void *stream);

/* --------------------------------------------------------- top level */
rg_status rg_tlas_sizes(int64_t n_inst, const rg_build_opts *opts, rg_sizes *out /*host*/);

/* The top level of the two-level structure, built from the instances'
 * transformation matrices (section 1: the second step, over the bottom
 * levels).  Builds the top level over n_inst instances.  blas: host array of
 * n_blas descriptors (all of the same width as opts); xform: host
 * float[n_inst][3][4] object->world, row-major; blas_id, inst_material: host
 * uint32[n_inst].  Instance boxes are the 8 transformed corners of the bottom
 * level's root box, computed in double and rounded outward to float; the
 * world->object inverse is computed in double and stored as float; a copy of
 * the matrices stays in out_buf (the trace calls recompute hits from it).
 * The bottom levels' root boxes are read from their headers on the device.
 * out_buf belongs to the caller and must outlive every trace and render over
 * it; the bottom levels must outlive it.  Synchronous: one upload of the host
 * tables and one wait (up to 4,096 instances build in one workgroup).  When
 * `stream` still has work queued, the upload goes on a stream of the
 * library's own (created with the first such call, per thread and device,
 * with an event and a device buffer of the tables' size that the library
 * keeps until the process ends) and `stream` waits for it just before the
 * build, so the copy overlaps the queued work.
 * Errors: RG_ERR_INVALID_ARG for NULL pointers, blas_id out of range, a
 * non-finite or singular matrix, mixed widths, or a bottom level whose last
 * refit found invalid input (its header's status word is set). */
rg_status rg_build_tlas(const rg_blas *blas, int32_t n_blas, const float *xform,
                        const uint32_t *blas_id, const uint32_t *inst_material, int64_t n_inst,
                        const rg_build_opts *opts, void *out_buf, uint64_t out_bytes,
                        void *scratch, uint64_t scratch_bytes, void *stream, rg_tlas *out /*host*/);

/* Top level with per-instance flags (host uint32[n_inst], nullable: every
 * instance RG_INST_MASK_ALL): bits 0-7 the visibility mask (a ray sees the
 * instance only if its own mask shares a bit with it; a mask of 0 hides the
 * instance from every ray, the render's included), RG_INST_CULL_DISABLE (face
 * culling never applies to its triangles), RG_INST_FLIP_FACING (front and back
 * exchange).  Other bits set: RG_ERR_INVALID_ARG.  Otherwise as
 * rg_build_tlas, which is this call with NULL. */
#define RG_INST_MASK_ALL 0xFFu
#define RG_INST_CULL_DISABLE (1u << 8)
#define RG_INST_FLIP_FACING (1u << 9)
rg_status rg_build_tlas_ex(const rg_blas *blas, int32_t n_blas, const float *xform,
                           const uint32_t *blas_id, const uint32_t *inst_material,
                           const uint32_t *inst_flags /*host, nullable*/, int64_t n_inst,
                           const rg_build_opts *opts, void *out_buf, uint64_t out_bytes,
                           void *scratch, uint64_t scratch_bytes, void *stream, rg_tlas *out /*host*/);

/* rg_build_tlas_ex without the wait (section 1's second step, enqueued), for
 * the linear builder (others: RG_ERR_UNSUPPORTED): everything the host
 * checks (as rg_build_tlas_ex) is checked and returned at once; the host
 * tables go to the device through the ticket, the build is enqueued on
 * `stream`, and rg_build_tlas_finish fills the descriptor.  ticket:
 * rg_tlas_ticket_bytes of pinned host memory (hipHostMalloc or a pinned
 * tensor), 256-byte aligned, owned by the caller; the bottom levels,
 * out_buf, scratch and the ticket must stay untouched until
 * rg_build_tlas_finish returns (the host arrays may be released when this
 * call returns). */
rg_status rg_tlas_ticket_bytes(int64_t n_inst, int32_t n_blas, int32_t with_flags, uint64_t *bytes /*host*/);
rg_status rg_build_tlas_async(const rg_blas *blas, int32_t n_blas, const float *xform,
                              const uint32_t *blas_id, const uint32_t *inst_material,
                              const uint32_t *inst_flags, int64_t n_inst, const rg_build_opts *opts,
                              void *out_buf, uint64_t out_bytes, void *scratch, uint64_t scratch_bytes,
                              void *stream, void *ticket /*pinned host*/, uint64_t ticket_bytes);

/* Completes an rg_build_tlas_async: waits until its stream has finished that
 * build, fills *out and returns its error (RG_ERR_INVALID_ARG for a bottom
 * level whose last refit found invalid input, or for a ticket that holds no
 * pending build: each completes once); a hierarchy deeper than the levels
 * the asynchronous call launched gets the rest here, with a wait. */
rg_status rg_build_tlas_finish(void *ticket /*pinned host*/, rg_tlas *out /*host*/);

/* ---------------------------------------------------------- tracing */
/* Closest hit for n rays (section 1: the closest-hit / miss outcome of each
 * ray against the two-level structure).  The traversal decides in float32,
 * with the watertight edge test, which triangle is hit; the reported t, u and
 * v are then recomputed for that triangle in double from the float32 inputs
 * (ray, instance matrix, vertices), so they carry no float32 cancellation
 * (t relative error ~1e-7 even for rays that start next to the surface);
 * t is clamped to [tmin, tmax], u and v to [0, 1].  Asynchronous.
 * Errors: RG_ERR_INVALID_ARG for NULL tlas/ray pointers, n < 0 (n == 0 is a
 * no-op) or t/u/v asked for without inst and prim; RG_ERR_UNSUPPORTED if the
 * hierarchy is deeper than the traversal stack holds (never for the
 * configurations built here). */
rg_status rg_trace_closest(const rg_tlas *tlas, rg_rays rays, int64_t n, rg_hits out, void *stream);

/* Any hit (section 1: the any-hit outcome; section 2.1: shadow rays):
 * occluded[i] = 1 if some triangle is hit in [tmin, tmax], else 0.  `found`
 * (nullable) receives one such hit (not necessarily the closest), its t, u, v
 * recomputed in double as for rg_trace_closest.  Asynchronous.  Errors as
 * rg_trace_closest. */
rg_status rg_trace_any(const rg_tlas *tlas, rg_rays rays, int64_t n, uint8_t *occluded,
                       const rg_hits *found /*host struct, nullable*/, void *stream);

/* Ray visibility and facing for the *_ex trace calls: the accept / ignore
 * decisions an any-hit stage makes in the paper's RTX model, in the form of
 * instance masks and cull flags.  A triangle faces the ray when the ray
 * travels against its winding normal (e1 x e2, e1 = v1 - v0, e2 = v2 - v0) in
 * the instance's object space (so a mirroring instance does not flip it;
 * RG_INST_FLIP_FACING does).  RG_RAY_CULL_BACK ignores triangles facing away
 * from the ray, RG_RAY_CULL_FRONT those facing it, except in instances flagged
 * RG_INST_CULL_DISABLE.  mask: the visibility mask of every ray (low 8 bits)
 * unless ray_mask (device uint8 per ray) is given.  NULL opts: no culling,
 * mask RG_INST_MASK_ALL (the plain calls).  Unknown flag bits or a mask above
 * 0xFF: RG_ERR_INVALID_ARG, checked on the host before anything is launched;
 * otherwise errors as the plain calls. */
#define RG_RAY_CULL_BACK 1u
#define RG_RAY_CULL_FRONT 2u
typedef struct {
    uint32_t flags;          /* RG_RAY_CULL_* */
    uint32_t mask;
    const uint8_t *ray_mask; /* device, nullable */
} rg_trace_opts;
rg_status rg_trace_closest_ex(const rg_tlas *tlas, rg_rays rays, int64_t n, rg_hits out,
                              const rg_trace_opts *opts /*host, nullable*/, void *stream);
rg_status rg_trace_any_ex(const rg_tlas *tlas, rg_rays rays, int64_t n, uint8_t *occluded,
                          const rg_hits *found /*host struct, nullable*/,
                          const rg_trace_opts *opts /*host, nullable*/, void *stream);

/* Visit counts per ray of the same traversal (closest if any_hit == 0):
 * counts uint32[n][3] = inner nodes, triangles, instances visited.  Used to
 * compute the bytes a traversal must move.  Asynchronous. */
rg_status rg_trace_counts(const rg_tlas *tlas, rg_rays rays, int64_t n, int32_t any_hit,
                          uint32_t *counts, void *stream);

/* Launch parameters of the traversal kernels, one set per family of calls
 * (process-wide):
 *   RG_TUNE_TRACE  rg_trace_closest, rg_trace_any, rg_trace_counts
 *   RG_TUNE_FRAME  rg_render, rg_batch_render
 *   RG_TUNE_ENGINE rg_engine_step
 * The kernels are persistent: the grid holds waves_per_cu waves per compute unit (at most
 * as many as the kernel variant keeps resident; defaults 20, 16 and 20), each
 * wave walks its own interleaved sequence of 64-ray packets, and its lanes
 * take new rays together once `refill` of them (1..64) are idle.  The first
 * lds_depth (8..32) entries of each lane's traversal stack live in LDS, the
 * rest in private memory.  A wave runs its leaf code once leaf_batch (1..64)
 * lanes wait at a leaf and its instance-entry code once inst_batch (1..64)
 * lanes wait at an instance (or when no lane has other work); 1 runs them
 * whenever any lane needs them.  Results do not depend on any of these.
 * Either pointer may be NULL.  Errors: RG_ERR_INVALID_ARG for an unknown
 * scope or values out of range. */
typedef struct {
    int32_t refill;
    int32_t waves_per_cu;
    int32_t lds_depth;
    int32_t leaf_batch;
    int32_t inst_batch;
} rg_trace_tune;
#define RG_TUNE_TRACE 0
#define RG_TUNE_FRAME 1
#define RG_TUNE_ENGINE 2
#define RG_TUNE_SCOPES 3
rg_status rg_trace_tuning(int32_t scope, const rg_trace_tune *set /*host, nullable*/,
                          rg_trace_tune *get /*host, nullable*/);

/* ---------------------------------------------------- ray generation */
/* The ray-generation step of a dispatch (section 1: a ray-generation shader
 * starts the rays of the frame): pinhole camera rays, one per pixel centre,
 * y = 0 the top row, vertical field of view: f = normalize(target-eye),
 * r = normalize(f x up), u = r x f, d = normalize(f + sx r + sy u), tmin = 0,
 * tmax = +inf.  Ray i is pixel i (row-major).  `rays` points to 8 device
 * float arrays (ox oy oz dx dy dz tmin tmax) of width*height entries, owned
 * by the caller.  Asynchronous.  Errors: RG_ERR_INVALID_ARG for a NULL
 * camera or array, width or height < 1, or more than 2^31 pixels. */
rg_status rg_camera_rays(const rg_camera *cam /*host*/, int32_t width, int32_t height,
                         float *const rays[8], void *stream);

/* Rays spawned at the hits of a first pass (section 1: a closest-hit
 * shader may spawn further rays), here the incoherent ambient-occlusion rays
 * of the measured workload: for each input ray i (n of them) whose hit is not
 * a miss, 8 cosine-weighted directions around the faced normal (Malley's
 * method in the Duff et al. 2017 basis), uniforms from SplitMix64 keyed by
 * (seed, i*8+k), origin offset 1e-4*max(1,|p|inf) along the faced normal,
 * tmin 0, tmax `ao_tmax`.  Output is compacted in input order: out_rays
 * (8 device float arrays of capacity 8n), out_src uint32[8n] = (i*8 + k), and
 * the count in *out_count (device uint32).  Asynchronous.  Errors:
 * RG_ERR_INVALID_ARG for NULL pointers or n < 0; RG_ERR_OUT_OF_MEMORY for
 * scratch shorter than rg_ao_rays_scratch. */
rg_status rg_ao_rays(const rg_tlas *tlas, rg_rays rays, int64_t n, const uint32_t *hit_inst,
                     const uint32_t *hit_prim, const float *hit_t, uint64_t seed, float ao_tmax,
                     float *const out_rays[8], uint32_t *out_src, uint32_t *out_count,
                     void *scratch, uint64_t scratch_bytes, void *stream);
rg_status rg_ao_rays_scratch(int64_t n, uint64_t *scratch_bytes /*host*/);

/* ------------------------------------------------------------ render */
/* Scratch bytes for rg_render at this size (host call). */
rg_status rg_render_sizes(int32_t width, int32_t height, int32_t max_depth, int32_t mode,
                          uint64_t *scratch_bytes /*host*/);

/* Renders one frame (section 1: rays spawned again by the shader a hit
 * invokes, each with its payload, to a bounded depth; section 2.1: shadow
 * casting, reflection and refraction on top of it): camera rays, then for
 * depth 0..max_depth a closest-hit pass, shading (sky on a miss; ambient term, a shadow ray towards the point
 * light for diffuse hits; a mirror child; reflection and refraction children
 * for glass with Schlick's Fresnel term, both spawned, none past max_depth),
 * an any-hit pass for the shadow rays and the direct term for unoccluded
 * ones.  mode 1 renders ambient occlusion instead (8 rays per primary hit,
 * tmax 5, pixel = 1 - occluded/8).  Contributions are summed per pixel in
 * 64-bit fixed point (scale 2^32), so the image does not depend on execution
 * order.  image: float[height][width][3], linear.  Asynchronous unless
 * `stats` is non-NULL (then it waits to fill it).
 * Errors: RG_ERR_INVALID_ARG (NULL pointers, sizes, max_depth > RG_MAX_DEPTH,
 * a material index out of range is not checked on the device: ids >= n_mats
 * are clamped), RG_ERR_OUT_OF_MEMORY (scratch too small). */
rg_status rg_render(const rg_tlas *tlas, const rg_material *mats /*host*/, int32_t n_mats,
                    const rg_camera *cam /*host*/, const rg_light *light /*host*/, int32_t width,
                    int32_t height, int32_t max_depth, int32_t mode, uint64_t seed, float *image,
                    void *scratch, uint64_t scratch_bytes, void *stream,
                    rg_render_stats *stats /*host, nullable*/);

/* rg_render that also writes, per pixel, the material its primary ray shaded
 * (the clamped material index; RG_MISS where the primary ray saw the sky)
 * to primary_mat (device uint32[height][width], nullable): the input of the
 * roughness blur below (section 2.1's screen-space roughness approximation).  primary_mat needs mode 0 (RG_ERR_UNSUPPORTED
 * otherwise). */
rg_status rg_render_ex(const rg_tlas *tlas, const rg_material *mats /*host*/, int32_t n_mats,
                       const rg_camera *cam /*host*/, const rg_light *light /*host*/, int32_t width,
                       int32_t height, int32_t max_depth, int32_t mode, uint64_t seed, float *image,
                       uint32_t *primary_mat, void *scratch, uint64_t scratch_bytes, void *stream,
                       rg_render_stats *stats /*host, nullable*/);

/* Trace parity inside a render (verification): rg_render (mode 0) that also
 * copies, after each pass k = 0..max_depth, that pass's queues to the caller:
 * the closest-hit rays exactly as traced (float32, origin and direction of
 * the secondary rays as spawned by shading), each one's float32 hit t and
 * its hit as input indices, and the shadow rays with their any-hit result.
 * So the traversal inside a render can be checked against an exact trace of
 * the very rays it traced, apart from the drift of secondary rays.  Buffers
 * (device): rays, shadow_rays float[max_depth + 1][8][capacity] (rows ox, oy,
 * oz, dx, dy, dz, tmin, tmax); t float, inst, prim uint32 and occluded uint8
 * [max_depth + 1][capacity]; counts uint32[max_depth + 1][2] = the pass's
 * queued closest-hit and shadow rays (only the first `capacity` of each are
 * copied).  The image is the same as rg_render's.  Asynchronous.
 * Errors: RG_ERR_INVALID_ARG for NULL capture buffers or capacity < 1,
 * otherwise as rg_render. */
typedef struct {
    int64_t capacity;
    float *rays, *t;
    uint32_t *inst, *prim;
    float *shadow_rays;
    uint8_t *occluded;
    uint32_t *counts;
} rg_capture;
rg_status rg_render_capture(const rg_tlas *tlas, const rg_material *mats /*host*/, int32_t n_mats,
                            const rg_camera *cam /*host*/, const rg_light *light /*host*/, int32_t width,
                            int32_t height, int32_t max_depth, uint64_t seed, float *image, void *scratch,
                            uint64_t scratch_bytes, const rg_capture *capture /*host*/, void *stream);

/* ------------------------------------------------------- post-process */
/* The frame's post-process passes (section 2.1: the engine's compute system
 * runs a screen-space roughness approximation and fast approximate
 * anti-aliasing on the traced image).  Images are device float[height][width]
 * [3] (the render's layout); input and output must not overlap, nor either
 * overlap the scratch buffer.  Asynchronous.  width * height <= 2^30. */

/* Scratch bytes for either pass (16 per pixel, rounded). */
rg_status rg_post_sizes(int32_t width, int32_t height, uint64_t *scratch_bytes /*host*/);

/* Material-aware Gaussian blur whose width follows the roughness of the
 * material seen at each pixel: two 1-D passes (along x, then y), each over
 * the taps k = -radius..radius with weights exp(-k^2 / (2 sigma^2)), sigma =
 * r radius / 3 (r = roughness[mat] clamped to [0, 1]); a tap counts if it lies
 * inside the image and shows the centre pixel's material; weights are
 * normalised over the taps that count.  Pixels whose material is RG_MISS,
 * >= n_mats or has roughness below 1/256 are copied.  mat: device
 * uint32[height][width]; roughness: device float[n_mats].
 * Errors: RG_ERR_INVALID_ARG (NULL pointers, sizes, radius outside
 * 0..RG_BLUR_RADIUS_MAX, overlapping buffers), RG_ERR_OUT_OF_MEMORY (scratch
 * below rg_post_sizes). */
#define RG_BLUR_RADIUS_MAX 16
rg_status rg_roughness_blur(const float *in, const uint32_t *mat, const float *roughness, int32_t n_mats,
                            int32_t width, int32_t height, int32_t radius, float *out, void *scratch,
                            uint64_t scratch_bytes, void *stream);

/* Fast approximate anti-aliasing (Lottes 2009, the "quality" variant) on the
 * perceptual luma sqrt(clamp(0.299 R + 0.587 G + 0.114 B, 0, 1)): edge
 * threshold max(1/16, 1/8 of the local maximum luma), edge search steps 1 (x5),
 * 1.5, 2 (x4), 4, 8 pixels each way, sub-pixel strength 3/4, clamp-to-edge.
 * Errors as rg_roughness_blur. */
rg_status rg_fxaa(const float *in, int32_t width, int32_t height, float *out, void *scratch,
                  uint64_t scratch_bytes, void *stream);

/* ------------------------------------------------------------ batches */
/* Many frames of different scenes and sizes rendered together, each the
 * render of rg_render (sections 1 and 2.1): every pass of the Whitted
 * recursion (closest hit, shading, shadow any hit, shadow resolve) is one
 * launch over the rays of all frames, each ray carrying its frame.  Each image is bitwise the one rg_render gives for the same frame.
 * All frames must use top levels of one width; mode must be 0. */
typedef struct {
    const rg_tlas *tlas;      /* host pointer to the frame's top level */
    const rg_material *mats;  /* host array of n_mats */
    int32_t n_mats;
    rg_camera cam;
    rg_light light;
    int32_t width, height, max_depth, mode;
    uint64_t seed;
    float *image;             /* device float[height][width][3] */
} rg_job;

/* Filled by rg_batch_prepare; describes the prepared scratch buffer. */
typedef struct {
    void *scratch;
    uint64_t scratch_bytes;
    int32_t n_jobs, width, max_depth, n_mats;
    int64_t total_pixels, capacity;
    int64_t cap_at[RG_MAX_DEPTH + 1]; /* queue bound per depth */
    int32_t has_inst_flags, reserved; /* some frame's top level carries instance flags */
} rg_batch;

/* Scratch bytes for a batch (host call).  Errors: RG_ERR_INVALID_ARG for a
 * bad frame, RG_ERR_UNSUPPORTED for mixed widths, mode 1 or more than 2^31
 * queue entries. */
rg_status rg_batch_sizes(const rg_job *jobs /*host*/, int32_t n_jobs, uint64_t *scratch_bytes /*host*/);

/* Copies the frame, top-level and material tables into `scratch` and fills
 * *out.  Synchronous: the host arrays may be released when it returns. */
rg_status rg_batch_prepare(const rg_job *jobs /*host*/, int32_t n_jobs, void *scratch, uint64_t scratch_bytes,
                           void *stream, rg_batch *out /*host*/);

/* Renders a prepared batch: kernel launches only, so a HIP graph can capture
 * it (then stats must be NULL).  Asynchronous unless stats is non-NULL. */
rg_status rg_batch_render(const rg_batch *batch /*host*/, void *stream, rg_render_stats *stats /*host, nullable*/);

/* ------------------------------------------------------------ serving */
/* The paper's renderer serves frames one dispatch at a time and keeps loaded
 * resources for reuse (section 2.2).  The engine below renders many frames
 * at once with continuous batching: it runs the Whitted recursion as passes
 * (closest hit, shading, shadow any hit, direct term) over the queued rays of
 * every frame in flight, each frame at its own depth.  A frame admitted
 * between passes queues its camera rays for the next pass; a frame leaves
 * after the pass at its max_depth, when its image is written.  Top levels,
 * bottom levels and images stay owned by the caller and must outlive the
 * frame.  Each image is bitwise the one rg_render gives for the same frame,
 * whatever else is in flight (64-bit fixed-point sums).
 *
 * Admission reserves, per frame, the queue entries one pass can hold for it
 * at worst (rg_job_reservation) and a contiguous range of pixel
 * accumulators; rg_pool is that accounting on its own (host only, no GPU
 * calls), for schedulers and tests.  Neither object is thread-safe. */
typedef struct rg_pool rg_pool;
typedef struct {
    int64_t rays, pixels, largest_free_pixels; /* reserved entries / pixels; largest free pixel range */
    int32_t jobs, reserved;                    /* frames holding a slot */
} rg_pool_usage;

/* A pool of max_rays queue entries (<= 2^31), max_pixels accumulator pixels
 * (<= 2^31) and max_jobs frame slots (<= 2^20).  Host call. */
rg_status rg_pool_create(int64_t max_rays, int64_t max_pixels, int32_t max_jobs, rg_pool **out /*host*/);
rg_status rg_pool_destroy(rg_pool *pool);
/* Reserves `rays` entries, `pixels` contiguous pixels (first fit) and the
 * lowest free slot.  *slot = -1 (RG_OK) when it does not fit now;
 * RG_ERR_OUT_OF_MEMORY when it could not fit an empty pool. */
rg_status rg_pool_reserve(rg_pool *pool, int64_t rays, int64_t pixels, int32_t *slot /*host*/,
                          int64_t *pix_off /*host*/);
/* Frees a slot's reservation (coalescing its pixel range). */
rg_status rg_pool_release(rg_pool *pool, int32_t slot);
rg_status rg_pool_get_usage(const rg_pool *pool, rg_pool_usage *out /*host*/);

/* Worst-case queue entries of one pass for a frame, and its pixels: a glass
 * hit spawns two children, a mirror hit one, a diffuse hit none, so a pass
 * at depth k holds at most width*height*2^k entries of a frame whose
 * materials include glass (width*height otherwise).  Host call. */
rg_status rg_job_reservation(const rg_job *job /*host*/, int64_t *rays /*host*/, int64_t *pixels /*host*/);

typedef struct {
    int64_t max_rays;   /* queue entries per pass (<= 2^31) */
    int64_t max_pixels; /* accumulator pixels of all frames in flight (<= 2^31) */
    int32_t max_jobs;   /* frames in flight */
    int32_t max_mats;   /* materials per frame */
    int32_t width;      /* node width of every top level admitted */
    int32_t reserved;
} rg_engine_desc;

typedef struct rg_engine rg_engine;
typedef struct {
    int64_t passes, passes_done;      /* passes enqueued / known complete */
    int64_t frames_live;              /* admitted, not yet returned by poll */
    int64_t frames_active;            /* with passes still to enqueue */
    int64_t admitted, completed;
    int64_t rays_reserved, pixels_reserved;
    int64_t max_frames_in_pass;       /* most frames sharing one pass so far */
    int64_t max_depths_in_pass;       /* most distinct recursion depths in one pass */
} rg_engine_info;

/* Scratch bytes of an engine (host call). */
rg_status rg_engine_sizes(const rg_engine_desc *desc /*host*/, uint64_t *scratch_bytes /*host*/);
/* Carves the engine's queues, accumulators and tables from `scratch` (the
 * library allocates no device memory) and enqueues their reset on `stream`;
 * every later call enqueues on the same stream. */
rg_status rg_engine_create(const rg_engine_desc *desc /*host*/, void *scratch, uint64_t scratch_bytes,
                           void *stream, rg_engine **out /*host*/);
/* Waits for the stream, then frees the host object. */
rg_status rg_engine_destroy(rg_engine *engine);
/* Admits a frame (mode 0) if its reservation fits: writes its record and
 * materials through kernel arguments (job->mats may go away on return),
 * zeroes its accumulators and queues its camera rays for the next pass.
 * Lifetime: the frame's top level, the bottom levels it refers to and its
 * image are read and written by the engine's passes (on its stream and a
 * side stream of its own) until rg_engine_poll returns the frame's tag; the
 * caller must keep them allocated until then (a caching allocator that
 * tracks streams does not see the engine's side stream).
 * *admitted = 0 when there is no room now (retry after a poll).  Errors:
 * RG_ERR_OUT_OF_MEMORY when the frame exceeds the whole engine,
 * RG_ERR_UNSUPPORTED for another node width or mode 1, RG_ERR_INVALID_ARG. */
rg_status rg_engine_admit(rg_engine *engine, const rg_job *job /*host*/, int64_t tag, int32_t *admitted /*host*/);
/* Enqueues one pass over every frame with passes left, and the image
 * resolve of the frames whose last pass it is.  *ran = 0 (nothing enqueued)
 * when no frame is active.  Blocks only when 32 passes are outstanding. */
rg_status rg_engine_step(rg_engine *engine, int32_t *ran /*host, nullable*/);
/* Returns up to `cap` tags of frames whose images are complete, in order of
 * completion, and frees their reservations.  wait != 0 first waits for the
 * oldest outstanding pass. */
rg_status rg_engine_poll(rg_engine *engine, int32_t wait, int64_t *tags /*host*/, int32_t cap,
                         int32_t *n_done /*host*/);
rg_status rg_engine_get_info(const rg_engine *engine, rg_engine_info *out /*host*/);
/* Rays traced since creation (closest-hit and shadow).  Synchronous. */
rg_status rg_engine_stats(rg_engine *engine, rg_render_stats *stats /*host*/);

/* ------------------------------------------------ build verification */
/* Runs the binary-hierarchy stages of rg_build_blas (with opts' builder;
 * opts NULL as for rg_build_blas) and copies their results out for
 * verification: keys uint64[n], the sorted Morton codes; ids uint32[n], the
 * triangle order of the leaves; left/right int32[n-1] of the binary
 * hierarchy (>= 0 inner node, < 0 leaf -(i+1), leaf i holding triangle
 * ids[i]; inner node 0 is the root); boxes float[2n-1][6] (inner nodes
 * 0..n-2, then the leaves 0..n-1).  For RG_BUILDER_LBVH the leaves are in
 * sorted order (ids = the sort's permutation); for RG_BUILDER_PLOC inner
 * nodes are numbered n-2 downward in merge order (a round's merges in order
 * of position) and the leaves are renumbered to the tree's left-to-right
 * order; for RG_BUILDER_TREELET the restructured linear BVH, its leaves
 * renumbered likewise.  scratch as for rg_build_blas.  Synchronous. */
rg_status rg_lbvh_stages(const float *verts, int64_t n_verts, const uint32_t *idx, int64_t n_tris,
                         const rg_build_opts *opts /*host, nullable*/, uint64_t *keys, uint32_t *ids,
                         int32_t *left, int32_t *right, float *boxes, void *scratch,
                         uint64_t scratch_bytes, void *stream);

/* ------------------------------------------ rendering without allocation */
/* rg_render for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * frame runs exactly as rg_render (image bitwise the same), with its scratch
 * in a device array of RG_STATIC_SCRATCH_BYTES inside the library (each GPU
 * holds one from the library's first use on it until the process ends), so
 * the caller passes only the inputs and the image, and the call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine; no stats, so
 * no events either).  Frames whose rg_render_sizes exceed the array are
 * refused with RG_ERR_OUT_OF_MEMORY before anything is enqueued (64 MiB holds
 * for instance 256x256 at depth 2, 128x128 at depth 4).  Every call on one
 * GPU uses that GPU's single array: calls that overlap on one GPU (other
 * streams, other threads) race, so serialise them; a call clears what it
 * needs cleared itself.  The first call on a device looks up the array's
 * address there (hipGetSymbolAddress).  Other errors as rg_render. */
#define RG_STATIC_SCRATCH_BYTES (64ull << 20)
rg_status rg_render_static(const rg_tlas *tlas, const rg_material *mats /*host*/, int32_t n_mats,
                           const rg_camera *cam /*host*/, const rg_light *light /*host*/, int32_t width,
                           int32_t height, int32_t max_depth, int32_t mode, uint64_t seed, float *image,
                           void *stream);

#ifdef __cplusplus
}
#endif
#endif /* RG_H */
