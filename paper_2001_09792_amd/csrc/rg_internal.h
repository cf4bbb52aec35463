// rg_internal.h -- types and helpers shared by the HIP translation units of
// librg.so.  Nothing here is part of the public ABI (include/rg.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rg.h"

#define RG_LEAF_BIT 0x80000000u
#define RG_EMPTY 0xFFFFFFFFu
#define RG_MAX_TRIS (1ll << 28)

// Leaf child encoding: bit 31 set, count-1 in bits 28..30, first in 0..27.
__host__ __device__ inline uint32_t rg_leaf(uint32_t first, uint32_t count) {
    return RG_LEAF_BIT | ((count - 1u) << 28) | first;
}
__host__ __device__ inline bool rg_is_leaf(uint32_t c) { return (c & RG_LEAF_BIT) != 0u; }
__host__ __device__ inline uint32_t rg_leaf_first(uint32_t c) { return c & 0x0FFFFFFFu; }
__host__ __device__ inline uint32_t rg_leaf_count(uint32_t c) { return ((c >> 28) & 7u) + 1u; }

// One `W`-wide node: child boxes as structure-of-arrays, then child links,
// padded to 32*W bytes so that a node is a whole number of 64-byte lines.
template <int W>
struct alignas(64) RgNode {
    float lo_x[W], lo_y[W], lo_z[W], hi_x[W], hi_y[W], hi_z[W];
    uint32_t child[W];
    uint32_t pad[W];
};
static_assert(sizeof(RgNode<2>) == 64, "node2");
static_assert(sizeof(RgNode<4>) == 128, "node4");
static_assert(sizeof(RgNode<8>) == 256, "node8");

// Triangle in leaf order: 40 bytes.
struct RgTri {
    float v[9];
    uint32_t prim;
};
static_assert(sizeof(RgTri) == 40, "tri");

// Header at the start of a bottom-level buffer (device addresses).
struct RgBlasHdr {
    uint64_t nodes, tris, mats, slots;
    float lo[3], hi[3];  // root box: written by the build and by every refit
    uint32_t status;     // flags of the last refit's input check (0: valid)
    uint32_t pad;
    uint64_t alpha;        // opacity masks, uint64 per input triangle (0: every triangle opaque)
    uint32_t alpha_level;  // micro-triangles per triangle: 4^alpha_level
    uint32_t pad2[13];
};
static_assert(sizeof(RgBlasHdr) == 128, "blas header");
static_assert(sizeof(rg_blas) == 120, "rg_blas layout (mirrored by the Python binding)");

// Instance record flag set by the top-level build when the instance's
// bottom level carries opacity masks (beside the caller's RG_INST_* bits).
#define RG_INST_ALPHA (1u << 16)

// Instance record in top-level leaf order: 112 bytes.
struct RgInst {
    float inv[9];  // world -> object linear part, row-major
    float p[3];    // object -> world translation (as given)
    uint64_t nodes, tris, hdr;
    uint32_t mat, inst;
    float blo[3], bhi[3];  // the bottom level's root box (object space)
    uint32_t flags;        // visibility mask (bits 0-7), RG_INST_CULL_DISABLE, RG_INST_FLIP_FACING, RG_INST_ALPHA
    uint32_t pad;
};
static_assert(sizeof(RgInst) == 112, "inst");

// Material as stored on the device.
struct RgMat {
    int32_t type;
    float rgb[3];
    float ior;
};
static_assert(sizeof(RgMat) == sizeof(rg_material), "material");

// Host-side error plumbing: the failing call is recorded per thread and
// reported by rg_last_error().
void rg_set_error(const char *file, int line, const char *what);

// With RG_DEBUG=1 in the environment (read once), an asynchronous entry point
// waits for its stream before returning and reports a failed launch or a
// device fault as RG_ERR_HIP; otherwise returns r unchanged.
rg_status rg_debug_done(rg_status r, hipStream_t st);
#define RG_HIP(x)                                                  \
    do {                                                           \
        hipError_t e_ = (x);                                       \
        if (e_ != hipSuccess) {                                    \
            rg_set_error(__FILE__, __LINE__, hipGetErrorName(e_)); \
            return RG_ERR_HIP;                                     \
        }                                                          \
    } while (0)
#define RG_LAUNCH_CHECK() RG_HIP(hipGetLastError())

// Bump allocator over a caller-provided buffer (256-byte granules).
struct RgArena {
    char *base;
    uint64_t size, used;
    template <class T>
    T *take(uint64_t count) {
        uint64_t bytes = (count * sizeof(T) + 255u) & ~uint64_t(255);
        if (base == nullptr) {  // sizing pass
            used += bytes;
            return nullptr;
        }
        if (used + bytes > size) {
            used += bytes;
            return nullptr;
        }
        T *p = reinterpret_cast<T *>(base + used);
        used += bytes;
        return p;
    }
    bool overflow() const { return base != nullptr && used > size; }
};

inline unsigned rg_blocks(int64_t n, int threads) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// Float <-> order-preserving uint32 (for atomic min/max of floats).
__device__ inline uint32_t rg_f2ord(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __host__ inline float rg_ord2f(uint32_t u) {
    uint32_t v = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
    float f;
    __builtin_memcpy(&f, &v, 4);
    return f;
}

// Shared LBVH build (build.hip), used by the bottom and the top level.
// prim_box: float[n][6] (lo xyz, hi xyz).  On success writes the wide nodes,
// the sorted primitive order (ids, in scratch), depth, node count and root box.
struct RgLbvhOut {
    uint32_t *ids;   // sorted primitive order (n)
    int32_t depth;
    int64_t n_nodes;
    float lo[3], hi[3];
    // Set by the caller to let a one-workgroup build (small n, linear BVH)
    // return without waiting: it then enqueues the copy of its summary
    // (depth, node count, error flag, root box: 10 uint32 / float words) to
    // *deferred and sets `pending`; the caller waits for the stream and calls
    // rg_lbvh_finish.
    uint32_t *deferred = nullptr;
    bool pending = false;
    const float *root_dev = nullptr;  // the root box (lo xyz, hi xyz) on the device, once the stream gets there
    // Optional device word that a one-workgroup build returns with its
    // summary (read when the build runs, after the caller's earlier steps on
    // the stream); rg_lbvh_finish stores it in `flag`.
    const uint32_t *flag_in = nullptr;
    uint32_t flag = 0;
    // Set by a larger build given `deferred`: the root box is on its way to
    // deferred[4..9]; rg_lbvh_finish (after the caller's wait) reads it.
    bool pending_box = false;
    // Set by the caller: 0 for 63-bit Morton keys, 33 for their top 30 bits
    // (ten per axis; four sort passes).
    int32_t key_shift = 0;
    // Set by an asynchronous caller (nullable): the multi-launch collapse
    // then launches its first batch of levels, records its state in
    // *coll_async and copies the level counts to coll_hr (pinned host) with
    // no wait; the caller completes it after the stream gets there.
    void *coll_async = nullptr;
    uint32_t *coll_hr = nullptr;
    // Set by the top-level build (nullable): a one-workgroup linear build of
    // up to 1,024 instances then also computes the instances' boxes and
    // records from the uploaded tables and writes the records in leaf order.
    const void *tlas_fuse = nullptr;
};
// Fills depth, n_nodes and the root box of a pending one-workgroup build
// from its summary (after the caller's wait); RG_ERR_HIP if it failed.
rg_status rg_lbvh_finish(RgLbvhOut *out, bool with_nodes);
// parents (nullable): per wide node, (parent node << 3) | slot in the parent,
// RG_MISS for the root.  levels (nullable, RG_LEVELS_CAP + 1 entries): the
// first node of each level and, after the last level, the node count (nodes
// are allocated level by level); left unwritten for deeper hierarchies.
rg_status rg_lbvh_build(const float *prim_box, int64_t n, int32_t width, int32_t leaf_max, int32_t builder,
                        int32_t radius, void *nodes, uint32_t *parents, uint32_t *levels, RgArena &scratch,
                        hipStream_t stream, RgLbvhOut *out, bool keep_stages, uint64_t *keys_out,
                        int32_t *left_out, int32_t *right_out, float *boxes_out);
uint64_t rg_lbvh_scratch_bytes(int64_t n, int32_t builder);

// In-place exclusive prefix sum of m uint32 values (one workgroup).
rg_status rg_scan_excl_u32(uint32_t *data, int64_t m, hipStream_t stream);
__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n);
