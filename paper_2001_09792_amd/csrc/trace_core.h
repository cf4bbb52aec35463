// trace_core.h -- the per-ray traversal of the two-level hierarchy, shared by
// the trace entry points and the render passes (both in trace.hip / render.hip).
//
// Per ray: test the W child boxes of the current node (robust slab test: the
// far distance is widened by 2*gamma_3, after Ize 2013, so rounding never
// drops a box the ray touches), continue with the nearest hit child and push
// the others far-to-near.  At a top-level leaf the ray is moved into the
// instance's object space: the ray is mapped with the world->object
// matrix in double (t is unchanged by the map), and its origin is slid to
// where it enters the bottom level's root box, so float32 coordinates stay
// box-sized; the slide t0 is added back to every t.  At a bottom-level leaf each
// triangle is tested with the watertight ray/triangle test of Woop, Benthin &
// Wald (JCGT 2013): vertices are sheared into ray space and three 2-D edge
// functions decide inside/outside; evaluated without fused multiply-add, a
// shared edge gives exactly negated values in its two triangles, so no ray
// passes between them.  Edges and vertices count as inside (two-sided,
// closed), a zero determinant (ray parallel to the plane) is a miss.
// Closest hit keeps the least t (ties: lowest instance, then primitive);
// any hit stops at the first triangle in [tmin, tmax].
#pragma once

#include "rg_internal.h"

namespace rgt {

constexpr int kThreads = 256;     // threads per workgroup of the trace kernels
constexpr int kMaxLdsStack = 32;  // most stack entries per lane kept in LDS (chosen per launch)
constexpr int kPrivStack = 96;    // further entries per lane in private memory
constexpr int kStackCap = 8 + kPrivStack;  // guaranteed capacity (at the smallest LDS depth, 8)
constexpr uint32_t kSentinel = 0xFFFFFFFEu;
constexpr uint32_t kFlip = 4u;  // in Tracer::cull: the instance flips its facing
// rounds a wave may run without any of its rays finishing: far above any
// traversal of a valid hierarchy (a loop bound, not a limit of the method)
constexpr uint32_t kMaxSteps = 1u << 22;
// The far distance of a slab is widened by 2 gamma_5 (gamma_n = n u / (1 - n u),
// u = 2^-24): the subtraction, the hardware reciprocal (1 ulp) and the product
// each add error to t, and the near distance may err the other way.
constexpr float kFarWiden = 2.0f * (5.0f * 5.9604645e-8f) / (1.0f - 5.0f * 5.9604645e-8f);
// Slab distances are computed as fma(plane, inv, -c): one rounding less in
// the relative error than (plane - o) * inv, but c = o * inv is rounded (by
// up to u |o inv|) and so is the shifted constant (u |c'|).  Shifting c by
// 3 u |o| |inv| (slightly more) towards the side that widens the slab keeps
// the lo-plane and hi-plane distances on the safe side of the exact ones.
constexpr float kSlabShift = 3.0f * 5.9604645e-8f * 1.01f;

#define RG_GLOBAL __attribute__((address_space(1)))
#define RG_LDS __attribute__((address_space(3)))

template <class T>
__device__ inline const RG_GLOBAL T *gptr(const void *p) {
    return (const RG_GLOBAL T *)(p);
}

typedef uint32_t rg_u4 __attribute__((ext_vector_type(4)));
typedef uint32_t rg_u2 __attribute__((ext_vector_type(2)));
typedef uint32_t rg_u4a8 __attribute__((ext_vector_type(4), aligned(8)));  // 16 bytes at 8-byte alignment

// Loads element i of a global array of T with global_load (T's size a
// multiple of 16 bytes and 16-byte aligned, or of 8 bytes for rg_u2 pieces).
template <class T, class V = rg_u4>
__device__ inline T gload(const void *base, uint64_t i) {
    static_assert(sizeof(T) % sizeof(V) == 0, "size");
    T out;
    const RG_GLOBAL V *src = (const RG_GLOBAL V *)((const char *)base + i * sizeof(T));
    V *dst = reinterpret_cast<V *>(&out);
#pragma unroll
    for (uint32_t k = 0; k < sizeof(T) / sizeof(V); ++k) dst[k] = src[k];
    return out;
}

enum Mode { kClosest = 0, kCounts = 1, kRender = 2 };
// Kinds of traversal unit.
constexpr uint32_t kUnitInner = 1, kUnitInst = 2, kUnitLeaf = 4;

struct Ray {
    float o[3], d[3], tmin, tmax;
};

// Result of one traversal: which triangle is hit.  For kRender `inst` is the
// top-level record index and `prim` the bottom-level triangle slot (leaf
// order); otherwise they are the input indices.  The hit's t is the
// tracer's `best` (closest hit); the trace entry points recompute t and the
// barycentrics of the chosen triangle in double afterwards (k_refine).
struct Hit {
    uint32_t inst, prim;
    uint32_t n_nodes, n_tris, n_inst;  // visit counts (kCounts)
};

__device__ inline float safe_rcp(float x) {
    // zero components get a huge finite reciprocal of the same sign, so that
    // (lo - o) * inv never evaluates 0 * inf; hardware reciprocal (1 ulp)
    const float tiny = 1e-30f;
    float y = fabsf(x) < tiny ? copysignf(tiny, x) : x;
    return __builtin_amdgcn_rcpf(y);
}

// Ray-space shear constants (Woop, Benthin & Wald 2013).
struct Shear {
    int kx, ky, kz;
    float sx, sy, sz;
};

__device__ inline Shear make_shear(const float d[3]) {
    Shear s;
    float ax = fabsf(d[0]), ay = fabsf(d[1]), az = fabsf(d[2]);
    s.kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    s.kx = s.kz == 2 ? 0 : s.kz + 1;
    s.ky = s.kx == 2 ? 0 : s.kx + 1;
    if (d[s.kz] < 0.0f) {
        int t = s.kx;
        s.kx = s.ky;
        s.ky = t;
    }
    // any consistent constants keep the test watertight: the same values
    // serve every triangle of the instance
    float rz = __builtin_amdgcn_rcpf(d[s.kz]);
    s.sx = d[s.kx] * rz;
    s.sy = d[s.ky] * rz;
    s.sz = rz;
    return s;
}

__device__ inline float comp(const float v[3], int k) { return k == 0 ? v[0] : (k == 1 ? v[1] : v[2]); }

// Watertight ray/triangle test in ray space.  Returns true on a hit whose
// t (in the ray's own frame) lies in [lo, hi] (up to a relative 1e-6 slack
// on either side, settled by the caller on the exact quotient), and writes
// T and det (t = T / det) and the edge values V, W (u = V / det, v = W / det).
// No division is done here: most triangles fail the edge or range test.
__device__ inline bool tri_test(const RgTri &tri, const float o[3], const Shear &s, float lo, float hi,
                                float &T_out, float &det_out, float &V_out, float &W_out) {
#pragma clang fp contract(off)
    const float *tv = tri.v;
    float a[3] = {tv[0] - o[0], tv[1] - o[1], tv[2] - o[2]};
    float b[3] = {tv[3] - o[0], tv[4] - o[1], tv[5] - o[2]};
    float c[3] = {tv[6] - o[0], tv[7] - o[1], tv[8] - o[2]};
    float az = comp(a, s.kz), bz = comp(b, s.kz), cz = comp(c, s.kz);
    float Ax = comp(a, s.kx) - s.sx * az, Ay = comp(a, s.ky) - s.sy * az;
    float Bx = comp(b, s.kx) - s.sx * bz, By = comp(b, s.ky) - s.sy * bz;
    float Cx = comp(c, s.kx) - s.sx * cz, Cy = comp(c, s.ky) - s.sy * cz;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    bool neg = (U < 0.0f) || (V < 0.0f) || (W < 0.0f);
    bool pos = (U > 0.0f) || (V > 0.0f) || (W > 0.0f);
    if (neg && pos) return false;
    float det = U + V + W;
    if (det == 0.0f) return false;
    float T = U * (s.sz * az) + V * (s.sz * bz) + W * (s.sz * cz);
    // range test without dividing: t in [lo, hi] <=> T in det*[lo, hi] for
    // det > 0 (reversed for det < 0); a small slack keeps it conservative
    float ad = fabsf(det), sT = det < 0.0f ? -T : T;
    float slack = 1e-6f * ad * fmaxf(fabsf(lo), fabsf(hi));
    if (sT > hi * ad + slack || sT < lo * ad - slack) return false;
    T_out = T;
    det_out = det;
    V_out = V;
    W_out = W;
    return true;
}

// Stack with the first n_lds entries in LDS (lane-interleaved, so the
// 64 lanes of a wave hit 64 different banks) and the rest in private memory.
struct Stack {
    uint32_t RG_LDS *lds;  // base of this lane's column: lds[e * kThreads]
    uint32_t *priv;        // kPrivStack further entries (a private array of the kernel)
    int sp;
    int n_lds;             // entries kept in LDS (8..kMaxLdsStack)
    __device__ inline void push(uint32_t v) {
        if (sp < n_lds) lds[sp * kThreads] = v;
        else priv[sp - n_lds] = v;
        ++sp;
    }
    __device__ inline uint32_t pop() {
        --sp;
        return sp < n_lds ? lds[sp * kThreads] : priv[sp - n_lds];
    }
    // Whether every active lane of the wave has m free LDS entries.
    __device__ inline bool room(int m) const { return __ballot(sp + m > n_lds) == 0ull; }
    // With room(): the entry goes to the top of the LDS part whether or not
    // it is kept; `keep` decides whether it stays (no branch per entry).
    __device__ inline void push_if(uint32_t v, bool keep) {
        lds[sp * kThreads] = v;
        sp += keep ? 1 : 0;
    }
};

template <int W>
__device__ inline void sort_children(float tn[W], uint32_t ch[W]) {
#define RG_CSWAP(i, j)                                  \
    if (tn[j] < tn[i]) {                                \
        float tf_ = tn[i]; tn[i] = tn[j]; tn[j] = tf_;  \
        uint32_t tc_ = ch[i]; ch[i] = ch[j]; ch[j] = tc_; \
    }
    if constexpr (W == 2) {
        RG_CSWAP(0, 1)
    } else if constexpr (W == 4) {
        RG_CSWAP(0, 1) RG_CSWAP(2, 3) RG_CSWAP(0, 2) RG_CSWAP(1, 3) RG_CSWAP(1, 2)
    } else {
        RG_CSWAP(0, 1) RG_CSWAP(2, 3) RG_CSWAP(4, 5) RG_CSWAP(6, 7)
        RG_CSWAP(0, 2) RG_CSWAP(1, 3) RG_CSWAP(4, 6) RG_CSWAP(5, 7)
        RG_CSWAP(1, 2) RG_CSWAP(5, 6) RG_CSWAP(0, 4) RG_CSWAP(3, 7)
        RG_CSWAP(1, 5) RG_CSWAP(2, 6)
        RG_CSWAP(1, 4) RG_CSWAP(3, 6)
        RG_CSWAP(2, 4) RG_CSWAP(3, 5)
        RG_CSWAP(3, 4)
    }
#undef RG_CSWAP
}

// Traversal of one ray as a resumable state machine: begin() loads the ray,
// step() performs one unit of work (an inner node, an instance entry, or a
// leaf's triangles, then the pop) and reports when the ray is finished.  The
// kernels run many rays per lane through it, so that lanes whose ray has
// finished can take a new one while the others continue.
// Opacity of the micro-triangle holding barycentrics (u, v) of a triangle cut
// into 4^level: cell (floor(n u), floor(n v)), n = 2^level, upright or
// inverted, numbered row by row (row j starts at j (2n - j)).
__device__ inline bool alpha_open(uint64_t mask, uint32_t level, float u, float v) {
    const int n = 1 << level;
    const float U = u * (float)n, V = v * (float)n;
    int i = (int)floorf(U), j = (int)floorf(V);
    i = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
    j = j < 0 ? 0 : (j > n - 1 - i ? n - 1 - i : j);
    const int inv = ((U - (float)i) + (V - (float)j) > 1.0f && i + j < n - 1) ? 1 : 0;
    return ((mask >> (j * (2 * n - j) + 2 * i + inv)) & 1ull) != 0ull;
}

// OPT: visibility masks, face culling and opacity masks are compiled in
// (launches whose rays carry options, or whose top levels carry instance
// flags or opacity masks); without it the traversal has none of their
// registers or tests.
template <int W, bool ANY, int MODE, bool OPT>
struct Tracer {
    const RgNode<W> *tlas_nodes;
    const RgInst *recs;
    Ray R;
    Hit h;
    float best;                 // closest: shrinks to the best hit (closed interval)
    float ox, oy, oz, ix, iy, iz;  // current frame: origin and reciprocal direction
    float t0, tlo, thi;         // slide of the frame's origin, interval in the frame
    const RgNode<W> *nodes;
    uint32_t tri_off;           // the bottom level's triangles: nodes + 16 tri_off bytes
    uint32_t inst_id;
    Shear sh;
    Stack st;
    uint32_t cur;
    uint32_t rmask;      // this ray's visibility mask
    uint32_t call_cull;  // RG_RAY_CULL_* of the launch
    uint32_t cull;       // culling in the current instance: RG_RAY_CULL_* | kFlip
    const uint64_t *alpha;  // opacity masks of the current instance's triangles (null: opaque)
    uint32_t alpha_level;
    bool in_blas, found;

    __device__ inline void world_frame() {
        in_blas = false;
        nodes = tlas_nodes;
        ox = R.o[0]; oy = R.o[1]; oz = R.o[2];
        ix = safe_rcp(R.d[0]); iy = safe_rcp(R.d[1]); iz = safe_rcp(R.d[2]);
        t0 = 0.0f;
        tlo = R.tmin;
        thi = best;
    }

    // Returns false if the ray has nothing to do (empty interval).
    __device__ inline bool begin(const Ray &ray) {
        R = ray;
        h.inst = h.prim = RG_MISS;
        h.n_nodes = h.n_tris = h.n_inst = 0;
        best = R.tmax;
        found = false;
        st.sp = 0;
        cur = 0;  // root inner node of the top level
        tri_off = 0u;
        inst_id = 0;
        sh.kx = 0; sh.ky = 1; sh.kz = 2; sh.sx = sh.sy = 0.0f; sh.sz = 1.0f;
        cull = 0u;
        alpha = nullptr;
        alpha_level = 0u;
        world_frame();
        return R.tmin <= R.tmax;
    }

    // Kind of the next unit: kUnitInner, kUnitInst or kUnitLeaf.
    __device__ inline uint32_t kind() const {
        return !rg_is_leaf(cur) ? kUnitInner : (!in_blas ? kUnitInst : kUnitLeaf);
    }

    // One unit of work; returns true when the ray is finished (h holds the
    // result, `found` whether there is a hit).
    //
    // Whatever the unit -- an inner node, an instance record or the first
    // two triangles of a leaf -- its bytes are requested before any of them
    // is used, into one register block, so that a wave whose lanes are at
    // different kinds of units waits for one memory round trip per step, not
    // one per kind (the three branches below run one after another under
    // divergence).  Leaves beyond two triangles load the rest as they go.
    // The caller decides which lanes run a unit this round.  The function has
    // one exit: early returns would each need their own copy of the whole
    // state at the merge after the call.
    __device__ inline bool step() {
        bool done = false;
        bool pop = false;
        constexpr int kNodeU4 = (7 * W + 3) / 4;  // node bytes without padding, in 16 B
        constexpr int kWords = 4 * kNodeU4 > 28 ? 4 * kNodeU4 : 28;
        const bool inner = !rg_is_leaf(cur);
        const bool inst = !inner && !in_blas;
        const uint32_t lf = rg_leaf_first(cur), ln = rg_leaf_count(cur);
        // The same load instructions serve every lane (only the address
        // differs), so no lane's load waits for another kind's.  112 bytes
        // cover a record, two triangles (a leaf of one reads into the next
        // triangle or the arrays after the last: every structure keeps at
        // least 112 bytes of its own buffer after each array) and a node of
        // width 2 or 4; width 8 nodes load their second half separately.
        const char *addr = inner ? (const char *)nodes + (uint64_t)cur * sizeof(RgNode<W>)
                                 : (inst ? (const char *)recs + (uint64_t)lf * sizeof(RgInst)
                                         : (const char *)nodes + 16ull * tri_off + (uint64_t)lf * sizeof(RgTri));
        uint32_t w[kWords];
        {
            const RG_GLOBAL rg_u4a8 *src = gptr<rg_u4a8>(addr);
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                const rg_u4a8 v = src[k];
                w[4 * k] = v.x; w[4 * k + 1] = v.y; w[4 * k + 2] = v.z; w[4 * k + 3] = v.w;
            }
            if (kNodeU4 > 7 && inner) {
#pragma unroll
                for (int k = 7; k < kNodeU4; ++k) {
                    const rg_u4a8 v = src[k];
                    w[4 * k] = v.x; w[4 * k + 1] = v.y; w[4 * k + 2] = v.z; w[4 * k + 3] = v.w;
                }
            }
        }
        const bool skip = OPT && inst && ((w[26] & 0xFFu) & rmask) == 0u;  // masked instance
        if (inner) {
            if (MODE == kCounts) ++h.n_nodes;
            float tn[W];
            uint32_t ch[W];
            // slab distances as one fused plane * inv - c each.  The constant
            // c of the lo planes and that of the hi planes sit on either side
            // of o * inv, kSlabShift |o| |inv| apart from it, on the side that
            // widens the slab whatever the sign of inv, so the rounding of
            // o * inv cannot narrow an interval; the far widening covers the
            // relative error as before
            float cl[3], chh[3];
            {
                const float o_[3] = {ox, oy, oz}, i_[3] = {ix, iy, iz};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const float c = o_[a] * i_[a], sh_ = kSlabShift * fabsf(o_[a]);
                    cl[a] = fmaf(sh_, i_[a], c);
                    chh[a] = fmaf(-sh_, i_[a], c);
                }
            }
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const float lx = __uint_as_float(w[k]), ly = __uint_as_float(w[W + k]);
                const float lz = __uint_as_float(w[2 * W + k]), hx = __uint_as_float(w[3 * W + k]);
                const float hy = __uint_as_float(w[4 * W + k]), hz = __uint_as_float(w[5 * W + k]);
                const float x0 = fmaf(lx, ix, -cl[0]), x1 = fmaf(hx, ix, -chh[0]);
                const float y0 = fmaf(ly, iy, -cl[1]), y1 = fmaf(hy, iy, -chh[1]);
                const float z0 = fmaf(lz, iz, -cl[2]), z1 = fmaf(hz, iz, -chh[2]);
                float n_ = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fmaxf(fminf(z0, z1), tlo));
                float f_ = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fmaxf(z0, z1));
                f_ = fmaf(fabsf(f_), kFarWiden, f_);
                f_ = fminf(f_, thi);
                ch[k] = w[6 * W + k];
                bool hit = (n_ <= f_) && (ch[k] != RG_EMPTY);
                tn[k] = hit ? n_ : INFINITY;
            }
            if (!ANY) sort_children<W>(tn, ch);
            // the nearest hit child continues; the others are pushed far first
            // (when the wave's LDS stacks have room for all of them: without
            // a branch per child)
            uint32_t next = RG_EMPTY;
            if (st.room(W - 1)) {  // wave-uniform
                if (ANY) {
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        const bool hk = tn[k] != INFINITY;
                        if (k > 0) st.push_if(ch[k], hk && next != RG_EMPTY);
                        next = (hk && next == RG_EMPTY) ? ch[k] : next;
                    }
                } else {
#pragma unroll
                    for (int k = W - 1; k >= 1; --k) st.push_if(ch[k], tn[k] != INFINITY);
                    next = tn[0] != INFINITY ? ch[0] : RG_EMPTY;
                }
            } else if (ANY) {
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    if (tn[k] != INFINITY) {
                        if (next == RG_EMPTY) next = ch[k];
                        else st.push(ch[k]);
                    }
                }
            } else {
#pragma unroll
                for (int k = W - 1; k >= 1; --k)
                    if (tn[k] != INFINITY) st.push(ch[k]);
                if (tn[0] != INFINITY) next = ch[0];
            }
            if (next != RG_EMPTY) cur = next;
            else pop = true;
        } else if (skip) {
            pop = true;  // not visible to this ray: as if missed
        } else if (inst) {
            // top-level leaf: one instance.  Record words: inv[9] 0..8, p[3]
            // 9..11, nodes 12..13, tris 14..15, hdr 16..17, mat 18, inst 19,
            // root box lo 20..22, hi 23..25, flags 26.
            if (MODE == kCounts) ++h.n_inst;
            // object-space ray in double: o' = M^-1 (o - p), d' = M^-1 d
            double q[3] = {(double)R.o[0] - (double)__uint_as_float(w[9]),
                           (double)R.o[1] - (double)__uint_as_float(w[10]),
                           (double)R.o[2] - (double)__uint_as_float(w[11])};
            double od[3], dd[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                double ir0 = __uint_as_float(w[3 * r]), ir1 = __uint_as_float(w[3 * r + 1]);
                double ir2 = __uint_as_float(w[3 * r + 2]);
                od[r] = ir0 * q[0] + ir1 * q[1] + ir2 * q[2];
                dd[r] = ir0 * (double)R.d[0] + ir1 * (double)R.d[1] + ir2 * (double)R.d[2];
            }
            // slide the origin to where the ray enters the bottom level's
            // root box (not before tmin); the entry only needs to be near the
            // box, so float suffices
            float ten = -INFINITY, tex = INFINITY;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                float of = (float)od[r], df = (float)dd[r], rr = safe_rcp(df);
                float a = (__uint_as_float(w[20 + r]) - of) * rr, b = (__uint_as_float(w[23 + r]) - of) * rr;
                ten = fmaxf(ten, fminf(a, b));
                tex = fminf(tex, fmaxf(a, b));
            }
            double ts = (ten <= tex && ten > R.tmin) ? (double)ten : (double)R.tmin;
            if (ts > (double)R.tmax) ts = (double)R.tmax;
            float t0f = (float)ts;
            float ld_[3];
            ox = (float)(od[0] + (double)t0f * dd[0]);
            oy = (float)(od[1] + (double)t0f * dd[1]);
            oz = (float)(od[2] + (double)t0f * dd[2]);
#pragma unroll
            for (int r = 0; r < 3; ++r) ld_[r] = (float)dd[r];
            ix = safe_rcp(ld_[0]); iy = safe_rcp(ld_[1]); iz = safe_rcp(ld_[2]);
            sh = make_shear(ld_);
            t0 = t0f;
            tlo = R.tmin - t0;
            tlo = tlo - fabsf(tlo) * 1.2e-7f;
            thi = best - t0;
            thi = thi + fabsf(thi) * 2.4e-7f;
            nodes = reinterpret_cast<const RgNode<W> *>((uint64_t)w[12] | ((uint64_t)w[13] << 32));
            // both arrays lie in the bottom level's buffer, 256-byte aligned,
            // the triangles after the nodes (at most 64 GB apart)
            tri_off = (uint32_t)((((uint64_t)w[14] | ((uint64_t)w[15] << 32)) -
                                  ((uint64_t)w[12] | ((uint64_t)w[13] << 32))) >> 4);
            inst_id = (MODE == kRender) ? lf : w[19];
            if (OPT) {
                cull = (w[26] & RG_INST_CULL_DISABLE) ? 0u : call_cull;
                if (cull && (w[26] & RG_INST_FLIP_FACING)) cull |= kFlip;
                alpha = nullptr;
                if (w[26] & RG_INST_ALPHA) {
                    const RgBlasHdr *H = reinterpret_cast<const RgBlasHdr *>((uint64_t)w[16] | ((uint64_t)w[17] << 32));
                    alpha = reinterpret_cast<const uint64_t *>(H->alpha);
                    alpha_level = H->alpha_level;
                }
            }
            in_blas = true;
            st.push(kSentinel);
            cur = 0;
        } else {
            // bottom-level leaf: up to 8 triangles, the first two already here
            const float o3[3] = {ox, oy, oz};
            bool stop = false;
            for (uint32_t j = 0; j < ln; ++j) {
                if (MODE == kCounts) ++h.n_tris;
                RgTri tri;
                if (j < 2) {
#pragma unroll
                    for (int k = 0; k < 9; ++k) tri.v[k] = __uint_as_float(j == 0 ? w[k] : w[10 + k]);
                    tri.prim = j == 0 ? w[9] : w[19];
                } else {
                    tri = gload<RgTri, rg_u2>((const char *)nodes + 16ull * tri_off, lf + j);
                }
                float T, det, V, Wv;
                if (!tri_test(tri, o3, sh, tlo, thi, T, det, V, Wv)) continue;
                if (OPT && cull) {
                    // facing: det > 0 when the ray travels against the winding
                    // normal (the sheared axes keep their handedness)
                    const bool front = (det > 0.0f) != ((cull & kFlip) != 0u);
                    if (cull & (front ? RG_RAY_CULL_FRONT : RG_RAY_CULL_BACK)) continue;
                }
                // t by the hardware reciprocal (1 ulp) and one product: up to
                // 1.5 ulp from T / det, inside the float32 band the parity
                // checks allow around t; the reported t is recomputed in double
                float tl = T * __builtin_amdgcn_rcpf(det);
                float tw = t0 + tl;
                if (!(tw >= R.tmin) || !(tw <= best)) continue;
                if (OPT && alpha && !alpha_open(alpha[tri.prim], alpha_level, V / det, Wv / det)) continue;
                uint32_t pid = (MODE == kRender) ? (lf + j) : tri.prim;
                if (!ANY && tw == best && found) {
                    if (inst_id > h.inst || (inst_id == h.inst && pid >= h.prim)) continue;
                }
                found = true;
                h.inst = inst_id;
                h.prim = pid;
                if (ANY) {
                    stop = true;
                    break;
                }
                best = tw;
                thi = best - t0;
                thi = thi + fabsf(thi) * 2.4e-7f;
            }
            if (stop) done = true;
            else pop = true;
        }
        if (pop) {
            // a sentinel (leaving an instance) is never directly above another
            if (st.sp == 0) {
                done = true;
            } else {
                uint32_t e = st.pop();
                if (e == kSentinel) {
                    world_frame();
                    if (st.sp == 0) done = true;
                    else e = st.pop();
                }
                cur = e;
            }
        }
        return done;
    }
};

}  // namespace rgt

// A top level as the kernels need it.
struct RgTlasRef {
    const void *nodes;
    const RgInst *recs;
};

// Arguments of the trace kernels (passed by value).
struct RgTraceArgs {
    const void *nodes;             // top-level nodes
    const RgInst *recs;            // top-level instance records
    const uint32_t *ray_job;       // per ray: index into jobs (nullable: all rays use nodes/recs)
    uint32_t ray_flags = 0u;       // RG_RAY_CULL_*
    uint32_t mask = RG_INST_MASK_ALL;  // visibility mask of every ray, unless ray_mask
    const uint8_t *ray_mask = nullptr;  // per ray (nullable)
    bool opt = false;              // masks / culling in effect (ray options or instance flags)
    const RgTlasRef *jobs;
    const float *ray[8];           // ox oy oz dx dy dz tmin tmax
    int64_t n;                     // number of rays (upper bound if `count` is set)
    const uint32_t *count;         // device count of rays (nullable)
    float *t, *u, *v;              // outputs (nullable)
    uint32_t *inst, *prim;
    uint8_t *occluded;             // any hit
    uint32_t *counts;              // visit counts [n][3]
    uint32_t *work;                // the launch's packet counters, two words (set by rg_trace_launch)
};

// Launches the traversal over a.n rays (or *a.count if set) on `stream`.
// width: 2/4/8; any: any-hit; mode: rgt::Mode.
// scope: the RG_TUNE_* family whose launch parameters apply.
rg_status rg_trace_launch(int width, bool any, int mode, const RgTraceArgs &a, hipStream_t stream, int scope);
// Compute units of the current device (queried once).
int rg_cu_count();
// Largest (W-1)*(top depth + bottom depth) + 1 the traversal stack holds.
bool rg_trace_depth_ok(const rg_tlas *t);
