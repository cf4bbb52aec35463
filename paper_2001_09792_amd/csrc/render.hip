// render.hip -- ray generation and the wavefront render loop.
//
// The paper's dispatch starts a ray-generation shader that casts the first
// rays; closest-hit / miss shaders then may spawn further rays, each carrying
// a payload, up to a recursion limit (section 1 and its footnote), and the
// render system adds reflection, refraction and shadow casting for multiple
// objects with material properties (section 2.1).  On gfx950 the recursion
// runs breadth-first: one pass per depth over a queue of rays whose payload
// is (pixel, throughput).  Shading adds the sky on a miss and the ambient
// term on a diffuse hit to the pixel, queues a shadow ray carrying the
// pending direct term, and queues mirror / glass children.  Children and
// shadow rays are appended with one atomic per wave (ballot + popcount
// ranks).  Pixel sums are 64-bit fixed point (2^32 per unit), so the image
// is independent of the order in which waves append and add.
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "wavefront.h"

namespace {

constexpr int kT = 256;
constexpr float kPi = 3.14159265358979323846f;

struct CamF {
    float eye[3], f[3], r[3], u[3], th;
};

__device__ inline void normalize3(float v[3]) {
    float l = sqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] = v[0] / l;
    v[1] = v[1] / l;
    v[2] = v[2] / l;
}
__device__ inline float dot3(const float a[3], const float b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
__device__ inline void cross3(float r[3], const float a[3], const float b[3]) {
    float x = a[1] * b[2] - a[2] * b[1], y = a[2] * b[0] - a[0] * b[2], z = a[0] * b[1] - a[1] * b[0];
    r[0] = x; r[1] = y; r[2] = z;
}

// Camera basis: f = normalize(target - eye), r = normalize(f x up), u = r x f.
__device__ inline CamF camera_basis(const rg_camera &c) {
    CamF k;
    float f[3] = {c.target[0] - c.eye[0], c.target[1] - c.eye[1], c.target[2] - c.eye[2]};
    normalize3(f);
    float r[3];
    cross3(r, f, c.up);
    normalize3(r);
    float u[3];
    cross3(u, r, f);
    for (int q = 0; q < 3; ++q) {
        k.eye[q] = c.eye[q]; k.f[q] = f[q]; k.r[q] = r[q]; k.u[q] = u[q];
    }
    k.th = tanf(0.5f * c.vfov_deg * (kPi / 180.0f));
    return k;
}

__device__ inline void camera_dir(const CamF &k, int W, int H, int64_t pixel, float d[3]) {
    int64_t x = pixel % W, y = pixel / W;
    float sx = (2.0f * ((float)x + 0.5f) / (float)W - 1.0f) * k.th * ((float)W / (float)H);
    float sy = (1.0f - 2.0f * ((float)y + 0.5f) / (float)H) * k.th;
    for (int q = 0; q < 3; ++q) d[q] = k.f[q] + sx * k.r[q] + sy * k.u[q];
    normalize3(d);
}

__global__ void k_camera_rays(rg_camera cam, int W, int H, float *o0, float *o1, float *o2, float *d0, float *d1,
                              float *d2, float *tmin, float *tmax) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t n = (int64_t)W * H;
    if (i >= n) return;
    CamF k = camera_basis(cam);
    float d[3];
    camera_dir(k, W, H, i, d);
    o0[i] = k.eye[0]; o1[i] = k.eye[1]; o2[i] = k.eye[2];
    d0[i] = d[0]; d1[i] = d[1]; d2[i] = d[2];
    tmin[i] = 0.0f;
    tmax[i] = INFINITY;
}

// ------------------------------------------------------ hit geometry
struct HitGeom {
    float p[3], ng[3], nf[3], dn[3];
    uint32_t mat;
};

__device__ inline void hit_geometry(const RgInst *recs, uint32_t rec_idx, uint32_t slot, const float o[3],
                                    const float d[3], float t, HitGeom &g) {
    const RgInst &R = recs[rec_idx];
    const RgTri tri = reinterpret_cast<const RgTri *>(R.tris)[slot];
    for (int q = 0; q < 3; ++q) g.p[q] = o[q] + t * d[q];
    float e1[3] = {tri.v[3] - tri.v[0], tri.v[4] - tri.v[1], tri.v[5] - tri.v[2]};
    float e2[3] = {tri.v[6] - tri.v[0], tri.v[7] - tri.v[1], tri.v[8] - tri.v[2]};
    float no[3];
    cross3(no, e1, e2);
    // normals map with the transpose of the world->object matrix
    float n[3];
    for (int c = 0; c < 3; ++c) n[c] = R.inv[c] * no[0] + R.inv[3 + c] * no[1] + R.inv[6 + c] * no[2];
    normalize3(n);
    for (int q = 0; q < 3; ++q) {
        g.ng[q] = n[q];
        g.dn[q] = d[q];
    }
    normalize3(g.dn);
    float s = dot3(g.ng, g.dn) < 0.0f ? 1.0f : -1.0f;
    for (int q = 0; q < 3; ++q) g.nf[q] = s * g.ng[q];
    if (R.mat != RG_PER_PRIM) {
        g.mat = R.mat;
    } else {
        const RgBlasHdr *h = reinterpret_cast<const RgBlasHdr *>(R.hdr);
        g.mat = reinterpret_cast<const uint16_t *>(h->mats)[slot];
    }
}

__device__ inline float offset_eps(const float p[3]) {
    float m = fmaxf(fmaxf(fabsf(p[0]), fabsf(p[1])), fabsf(p[2]));
    return 1e-4f * fmaxf(1.0f, m);
}

// ------------------------------------------------------ fixed point
__device__ inline void accum_add(unsigned long long *acc, uint32_t pixel, const float v[3]) {
    for (int q = 0; q < 3; ++q) {
        if (!(v[q] > 0.0f)) continue;
        unsigned long long x = (unsigned long long)llrint((double)v[q] * 4294967296.0);
        atomicAdd(acc + 3 * (uint64_t)pixel + q, x);
    }
}

// --------------------------------------------------------- queues
__device__ inline void put_ray(float *const ray[8], uint32_t j, const float o[3], const float d[3], float tmin,
                               float tmax) {
    ray[0][j] = o[0]; ray[1][j] = o[1]; ray[2][j] = o[2];
    ray[3][j] = d[0]; ray[4][j] = d[1]; ray[5][j] = d[2];
    ray[6][j] = tmin; ray[7][j] = tmax;
}

// Appends `cnt` (0..2) entries per lane with one atomic per wave; returns
// this lane's first slot.
__device__ inline uint32_t wave_append(uint32_t *counter, uint32_t cnt) {
    uint64_t b1 = __ballot(cnt >= 1u), b2 = __ballot(cnt >= 2u);
    int lane = threadIdx.x & 63;
    uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint32_t before = (uint32_t)(__popcll(b1 & lt) + __popcll(b2 & lt));
    uint32_t total = (uint32_t)(__popcll(b1) + __popcll(b2));
    uint64_t active = __ballot(1);
    int leader = __ffsll((long long)active) - 1;
    uint32_t base = 0;
    if (lane == leader && total > 0) base = atomicAdd(counter, total);
    base = __shfl(base, leader, 64);
    return base + before;
}

// Block-wide append of two counts per thread (0..2 to `a`, 0..1 to `b`):
// ballot ranks inside each wave, wave totals in LDS, one atomic per counter
// per block.  Every thread of the block must call it.
constexpr int kShadeT = 512;
__device__ inline void block_append2(uint32_t *ctr_a, uint32_t cnt_a, uint32_t *ctr_b, uint32_t cnt_b,
                                     uint32_t &pos_a, uint32_t &pos_b) {
    constexpr int NW = kShadeT / 64;
    __shared__ uint32_t wa[NW], wb[NW], base[2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint64_t a1 = __ballot(cnt_a >= 1u), a2 = __ballot(cnt_a >= 2u), b1 = __ballot(cnt_b >= 1u);
    const uint32_t ra = (uint32_t)(__popcll(a1 & lt) + __popcll(a2 & lt)), rb = (uint32_t)__popcll(b1 & lt);
    if (lane == 0) {
        wa[w] = (uint32_t)(__popcll(a1) + __popcll(a2));
        wb[w] = (uint32_t)__popcll(b1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t sa = 0, sb = 0;
        for (int k = 0; k < NW; ++k) {
            uint32_t ta = wa[k], tb = wb[k];
            wa[k] = sa;
            wb[k] = sb;
            sa += ta;
            sb += tb;
        }
        base[0] = sa ? atomicAdd(ctr_a, sa) : 0u;
        base[1] = sb ? atomicAdd(ctr_b, sb) : 0u;
    }
    __syncthreads();
    pos_a = base[0] + wa[w] + ra;
    pos_b = base[1] + wb[w] + rb;
    __syncthreads();  // the next call may overwrite the LDS
}

// The frame owning accumulator index p (frames are stored in pix_off order).
__device__ inline uint32_t find_job(const RgJobDev *jobs, int n_jobs, uint32_t p) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].pix_off <= p) lo = mid;
        else hi = mid - 1;
    }
    return (uint32_t)lo;
}

__global__ void k_camera_batch(const RgJobDev *__restrict__ jobs, int n_jobs, int64_t total, RgQueue q,
                               uint32_t *count) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i == 0) *count = (uint32_t)total;
    if (i >= total) return;
    uint32_t j = find_job(jobs, n_jobs, (uint32_t)i);
    const RgJobDev &J = jobs[j];
    CamF k = camera_basis(J.cam);
    float d[3];
    camera_dir(k, (int)J.width, (int)J.height, i - J.pix_off, d);
    float o[3] = {k.eye[0], k.eye[1], k.eye[2]};
    put_ray(q.ray, (uint32_t)i, o, d, 0.0f, INFINITY);
    q.pix[i] = (uint32_t)i;
    q.job[i] = j;
    q.beta[0][i] = 1.0f;
    q.beta[1][i] = 1.0f;
    q.beta[2][i] = 1.0f;
}

struct ShadeArgs {
    RgQueue in;
    const uint32_t *count_in;
    const float *hit_t;
    const uint32_t *hit_rec, *hit_slot;
    const RgTlasRef *tlas;  // per job
    const RgJobDev *jobs;
    const RgMat *mats;      // all jobs' materials, job j's at jobs[j].mat_off
    int64_t pass;           // entry depth = pass - jobs[job].start
    unsigned long long *acc;
    RgQueue out;
    uint32_t *count_out;
    RgShadowQ sq;
    uint32_t *count_sq;
    int64_t cap_out, cap_sq;
    int64_t n_max;          // entries the input queue can hold
};

// Persistent: blocks stride over the queue; each round of kShadeT entries
// appends its children and shadow rays with one atomic per counter.
__global__ void __launch_bounds__(kShadeT) k_shade(ShadeArgs a) {
    const int64_t n = (int64_t)*a.count_in < a.n_max ? (int64_t)*a.count_in : a.n_max;
    for (int64_t base = (int64_t)blockIdx.x * kShadeT; base < n; base += (int64_t)gridDim.x * kShadeT) {
    const int64_t i = base + threadIdx.x;
    const bool active = i < n;
    uint32_t n_child = 0, n_shadow = 0;
    float co[2][3], cd[2][3], cb[2][3];
    float so[3], sd[3], sp[3];
    uint32_t pixel = 0, job = 0;
    if (active) {
        pixel = a.in.pix[i];
        job = a.in.job[i];
        float beta[3] = {a.in.beta[0][i], a.in.beta[1][i], a.in.beta[2][i]};
        float o[3] = {a.in.ray[0][i], a.in.ray[1][i], a.in.ray[2][i]};
        float d[3] = {a.in.ray[3][i], a.in.ray[4][i], a.in.ray[5][i]};
        uint32_t rec = a.hit_rec[i];
        const bool primary = a.pass == a.jobs[job].start;
        uint32_t *gbuf = primary ? a.jobs[job].gbuf : nullptr;
        if (rec == RG_MISS) {
            if (gbuf) gbuf[pixel - a.jobs[job].pix_off] = RG_MISS;
            float dn[3] = {d[0], d[1], d[2]};
            normalize3(dn);
            float s = 0.5f * (dn[1] + 1.0f);
            float sky[3] = {(1.0f - s) + s * 0.5f, (1.0f - s) + s * 0.7f, (1.0f - s) + s * 1.0f};
            float v[3] = {beta[0] * sky[0], beta[1] * sky[1], beta[2] * sky[2]};
            accum_add(a.acc, pixel, v);
        } else {
            const RgJobDev &J = a.jobs[job];
            HitGeom g;
            hit_geometry(a.tlas[job].recs, rec, a.hit_slot[i], o, d, a.hit_t[i], g);
            uint32_t mid = g.mat < J.n_mats ? g.mat : J.n_mats - 1;
            if (gbuf) gbuf[pixel - J.pix_off] = mid;
            const RgMat M = a.mats[J.mat_off + mid];
            float eps = offset_eps(g.p);
            if (M.type == 0) {
                float amb[3] = {beta[0] * M.rgb[0] * J.light.ambient, beta[1] * M.rgb[1] * J.light.ambient,
                                beta[2] * M.rgb[2] * J.light.ambient};
                accum_add(a.acc, pixel, amb);
                float l[3] = {J.light.pos[0] - g.p[0], J.light.pos[1] - g.p[1], J.light.pos[2] - g.p[2]};
                normalize3(l);
                float c = dot3(g.nf, l);
                if (c > 0.0f) {
                    n_shadow = 1;
                    for (int q = 0; q < 3; ++q) {
                        so[q] = g.p[q] + eps * g.nf[q];
                        sd[q] = J.light.pos[q] - so[q];
                        sp[q] = beta[q] * M.rgb[q] * J.light.intensity[q] * c;
                    }
                }
            } else if (a.pass - J.start < (int64_t)J.max_depth) {
                float dnf = dot3(g.dn, g.nf);
                for (int q = 0; q < 3; ++q) {
                    co[0][q] = g.p[q] + eps * g.nf[q];
                    cd[0][q] = g.dn[q] - 2.0f * dnf * g.nf[q];
                }
                if (M.type == 1) {
                    n_child = 1;
                    for (int q = 0; q < 3; ++q) cb[0][q] = beta[q] * M.rgb[q];
                } else {
                    bool entering = dot3(g.dn, g.ng) < 0.0f;
                    float ior = M.ior;
                    float eta = entering ? 1.0f / ior : ior;
                    float cosi = -dnf;
                    float kappa = 1.0f - eta * eta * (1.0f - cosi * cosi);
                    if (kappa < 0.0f) {
                        n_child = 1;
                        for (int q = 0; q < 3; ++q) cb[0][q] = beta[q];
                    } else {
                        float sk = sqrtf(kappa);
                        float r0 = (ior - 1.0f) / (ior + 1.0f);
                        r0 = r0 * r0;
                        float cc = entering ? cosi : sk;
                        float om = 1.0f - cc;
                        float F = r0 + (1.0f - r0) * om * om * om * om * om;
                        n_child = 2;
                        for (int q = 0; q < 3; ++q) {
                            cb[0][q] = beta[q] * F;
                            co[1][q] = g.p[q] - eps * g.nf[q];
                            cd[1][q] = eta * g.dn[q] + (eta * cosi - sk) * g.nf[q];
                            cb[1][q] = beta[q] * (1.0f - F);
                        }
                    }
                }
            }
        }
    }
    uint32_t cs, ss;
    block_append2(a.count_out, n_child, a.count_sq, n_shadow, cs, ss);
    for (uint32_t c = 0; c < n_child; ++c) {
        uint32_t j = cs + c;
        if ((int64_t)j >= a.cap_out) break;  // the queue holds sum n 2^D entries: never reached
        put_ray(a.out.ray, j, co[c], cd[c], 0.0f, INFINITY);
        a.out.pix[j] = pixel;
        a.out.job[j] = job;
        a.out.beta[0][j] = cb[c][0];
        a.out.beta[1][j] = cb[c][1];
        a.out.beta[2][j] = cb[c][2];
    }
    if (n_shadow && (int64_t)ss < a.cap_sq) {
        put_ray(a.sq.ray, ss, so, sd, 0.0f, 1.0f - 1e-4f);
        a.sq.pix[ss] = pixel;
        a.sq.job[ss] = job;
        a.sq.pend[0][ss] = sp[0];
        a.sq.pend[1][ss] = sp[1];
        a.sq.pend[2][ss] = sp[2];
    }
    }
}

__global__ void k_shadow_resolve(RgShadowQ sq, const uint32_t *count, unsigned long long *acc) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)*count) return;
    if (sq.occ[i]) return;
    float v[3] = {sq.pend[0][i], sq.pend[1][i], sq.pend[2][i]};
    accum_add(acc, sq.pix[i], v);
}

__global__ void k_resolve_batch(const unsigned long long *acc, const RgJobDev *__restrict__ jobs, int n_jobs,
                                int64_t total) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= total) return;
    const RgJobDev &J = jobs[find_job(jobs, n_jobs, (uint32_t)i)];
    int64_t local = i - J.pix_off;
    for (int c = 0; c < 3; ++c) J.image[3 * local + c] = (float)((double)acc[3 * i + c] * (1.0 / 4294967296.0));
}

__global__ void k_zero_u64(unsigned long long *p, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void k_stat_add(unsigned long long *stat, const uint32_t *count) { *stat += *count; }

// Between a pass's closest-hit launch and its shading: the rays it traced
// go into the statistics, and the next pass's queue count and the shadow
// queue count start at zero (one launch instead of three).
__global__ void k_pass_counts(unsigned long long *stat, const uint32_t *count_in, uint32_t *count_out,
                              uint32_t *count_shadow) {
    *stat += *count_in;
    *count_out = 0u;
    *count_shadow = 0u;
}

// Frame record and materials written through kernel arguments: nothing
// for the host to keep alive, nothing to wait for, capturable.
__global__ void k_put_job(RgJobDev *jobs, RgTlasRef *tlas, uint32_t slot, RgJobDev J, RgTlasRef T) {
    if (threadIdx.x == 0) {
        jobs[slot] = J;
        tlas[slot] = T;
    }
}

constexpr int kMatChunk = 64;
struct MatChunk {
    RgMat m[kMatChunk];
};
__global__ void k_put_mats(RgMat *dst, MatChunk c, int n) {
    if ((int)threadIdx.x < n) dst[threadIdx.x] = c.m[threadIdx.x];
}

// Reserves n consecutive queue entries for a frame's camera rays: *base =
// old count.
__global__ void k_reserve(uint32_t *count, uint32_t n, uint32_t *base) {
    if (threadIdx.x == 0) *base = atomicAdd(count, n);
}

// One camera ray per pixel of frame `slot`, at *base + pixel.
__global__ void __launch_bounds__(kT) k_camera_job(RgJobDev J, uint32_t slot, RgQueue q, const uint32_t *base,
                                                   int64_t cap) {
    int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x;
    const int64_t n = (int64_t)J.width * J.height;
    const int64_t at = (int64_t)*base + i;
    if (i >= n || at >= cap) return;
    CamF k = camera_basis(J.cam);
    float d[3];
    camera_dir(k, (int)J.width, (int)J.height, i, d);
    float o[3] = {k.eye[0], k.eye[1], k.eye[2]};
    put_ray(q.ray, at, o, d, 0.0f, INFINITY);
    q.pix[at] = J.pix_off + (uint32_t)i;
    q.job[at] = slot;
    q.beta[0][at] = 1.0f;
    q.beta[1][at] = 1.0f;
    q.beta[2][at] = 1.0f;
}

__global__ void k_resolve_job(const unsigned long long *acc, int64_t n, float *image) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= 3 * n) return;
    image[i] = (float)((double)acc[i] * (1.0 / 4294967296.0));
}

// -------------------------------------------------- ambient occlusion
__device__ inline uint64_t splitmix_out(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Cosine-weighted direction around unit n (Malley's method) in the basis of
// Duff et al. 2017; uniforms from SplitMix64 started at seed + 2 key gamma.
__device__ inline void ao_dir(const float n[3], uint64_t seed, uint64_t key, float out[3]) {
    const uint64_t g = 0x9E3779B97F4A7C15ull;
    uint64_t s = seed + 2ull * key * g;
    float u1 = (float)(splitmix_out(s + g) >> 40) * (1.0f / 16777216.0f);
    float u2 = (float)(splitmix_out(s + 2ull * g) >> 40) * (1.0f / 16777216.0f);
    float sgn = n[2] >= 0.0f ? 1.0f : -1.0f;
    float a = -1.0f / (sgn + n[2]);
    float b = n[0] * n[1] * a;
    float b1[3] = {1.0f + sgn * n[0] * n[0] * a, sgn * b, -sgn * n[0]};
    float b2[3] = {b, sgn + n[1] * n[1] * a, -n[1]};
    float r = sqrtf(u1);
    float sp, cp;
    sincospif(2.0f * u2, &sp, &cp);
    float x = r * cp, y = r * sp, z = sqrtf(1.0f - u1);
    for (int q = 0; q < 3; ++q) out[q] = x * b1[q] + y * b2[q] + z * n[q];
}

struct AoArgs {
    const float *ray[8];
    int64_t n;
    const uint32_t *hit_a, *hit_b;  // (rec, slot), or (inst, prim) input ids if map
    const float *hit_t;
    const uint32_t *rec_of;         // tlas: record of an input instance (map only)
    const RgInst *recs;
    uint64_t seed;
    float tmax;
    float *out[8];
    uint32_t *src;
    uint32_t *count;
    uint32_t *block_off;            // per-block offsets (scanned)
    bool map;
};

__device__ inline bool ao_hit(const AoArgs &a, int64_t i) { return i < a.n && a.hit_a[i] != RG_MISS; }

__global__ void k_ao_count(AoArgs a) {
    int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x;
    uint64_t b = __ballot(ao_hit(a, i));
    __shared__ uint32_t wc[kT / 64];
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = (uint32_t)__popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kT / 64; ++w) s += wc[w];
        a.block_off[blockIdx.x] = 8u * s;
    }
}

__global__ void k_ao_emit(AoArgs a, int nblocks, const uint32_t *block_cnt_last) {
    int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x;
    bool h = ao_hit(a, i);
    uint64_t b = __ballot(h);
    __shared__ uint32_t wc[kT / 64];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) wc[w] = (uint32_t)__popcll(b);
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int q = 0; q < kT / 64; ++q) {
        if (q < w) before += wc[q];
        tot += wc[q];
    }
    uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    before += (uint32_t)__popcll(b & lt);
    uint32_t base = a.block_off[blockIdx.x];
    if (blockIdx.x == (unsigned)(nblocks - 1) && threadIdx.x == 0) *a.count = base + 8u * tot;
    if (!h) return;
    uint32_t rec = a.hit_a[i], slot = a.hit_b[i];
    if (a.map) {
        rec = a.rec_of[rec];
        const RgBlasHdr *hd = reinterpret_cast<const RgBlasHdr *>(a.recs[rec].hdr);
        slot = reinterpret_cast<const uint32_t *>(hd->slots)[slot];
    }
    float o[3] = {a.ray[0][i], a.ray[1][i], a.ray[2][i]};
    float d[3] = {a.ray[3][i], a.ray[4][i], a.ray[5][i]};
    HitGeom g;
    hit_geometry(a.recs, rec, slot, o, d, a.hit_t[i], g);
    float eps = offset_eps(g.p);
    float org[3] = {g.p[0] + eps * g.nf[0], g.p[1] + eps * g.nf[1], g.p[2] + eps * g.nf[2]};
    uint32_t j0 = base + 8u * before;
    for (int k = 0; k < 8; ++k) {
        float dir[3];
        ao_dir(g.nf, a.seed, (uint64_t)i * 8ull + (uint64_t)k, dir);
        put_ray(a.out, j0 + k, org, dir, 0.0f, a.tmax);
        a.src[j0 + k] = (uint32_t)(i * 8 + k);
    }
}

__global__ void k_ao_accum(const uint8_t *occ, const uint32_t *src, const uint32_t *count,
                           unsigned long long *acc) {
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= (int64_t)*count) return;
    if (occ[j]) atomicAdd(acc + 3 * (uint64_t)(src[j] >> 3), 1ull);
}

__global__ void k_ao_resolve(const unsigned long long *acc, const uint32_t *hit_rec, int64_t n, float *image) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v = 1.0f;
    if (hit_rec[i] != RG_MISS) v = 1.0f - (float)acc[3 * i] * 0.125f;
    image[3 * i] = v;
    image[3 * i + 1] = v;
    image[3 * i + 2] = v;
}

rg_status ao_generate(AoArgs a, hipStream_t st) {
    int nb = (int)rg_blocks(a.n, kT);
    k_ao_count<<<nb, kT, 0, st>>>(a);
    RG_LAUNCH_CHECK();
    rg_status r = rg_scan_excl_u32(a.block_off, nb, st);
    if (r != RG_OK) return r;
    k_ao_emit<<<nb, kT, 0, st>>>(a, nb, nullptr);
    RG_LAUNCH_CHECK();
    return RG_OK;
}

// ------------------------------------------------------ scratch layout
// ambient occlusion (one frame)
struct AoBufs {
    unsigned long long *acc, *stat;
    uint32_t *counts;
    float *hit_t;
    uint32_t *hit_rec, *hit_slot;
    float *cam[8];
    float *ao_ray[8];
    uint32_t *ao_src, *ao_blk;
    uint8_t *ao_occ;
};

bool carve_ao(RgArena &A, int64_t n, AoBufs &b) {
    b.acc = A.take<unsigned long long>(3 * n);
    b.stat = A.take<unsigned long long>(4);
    b.counts = A.take<uint32_t>(8);
    b.hit_t = A.take<float>(n);
    b.hit_rec = A.take<uint32_t>(n);
    b.hit_slot = A.take<uint32_t>(n);
    for (int c = 0; c < 8; ++c) b.cam[c] = A.take<float>(n);
    for (int c = 0; c < 8; ++c) b.ao_ray[c] = A.take<float>(8 * n);
    b.ao_src = A.take<uint32_t>(8 * n);
    b.ao_blk = A.take<uint32_t>(rg_blocks(n, kT));
    b.ao_occ = A.take<uint8_t>(8 * n);
    return !A.overflow();
}

bool tlas_valid(const rg_tlas *t) {
    return t && t->buf && t->n_inst >= 1 && (t->width == 2 || t->width == 4 || t->width == 8);
}

RgTraceArgs trace_args(const rg_tlas *t) {
    RgTraceArgs a = {};
    a.nodes = (const char *)t->buf + t->nodes_off;
    a.recs = (const RgInst *)((const char *)t->buf + t->inst_off);
    a.opt = t->has_inst_flags != 0;
    return a;
}

struct BatchShape {
    int64_t total_pix = 0, cap = 0;
    int64_t cap_at[RG_MAX_DEPTH + 1] = {};
    int32_t n_mats = 0, max_depth = 0, width = 0;
};

rg_status batch_shape(const rg_job *jobs, int32_t n_jobs, BatchShape &sh) {
    if (!jobs || n_jobs < 1 || n_jobs > (1 << 20)) return RG_ERR_INVALID_ARG;
    for (int32_t j = 0; j < n_jobs; ++j) {
        const rg_job &J = jobs[j];
        if (!tlas_valid(J.tlas) || !J.mats || J.n_mats < 1 || J.n_mats > 65536 || !J.image) return RG_ERR_INVALID_ARG;
        if (J.width < 1 || J.height < 1 || J.max_depth < 0 || J.max_depth > RG_MAX_DEPTH) return RG_ERR_INVALID_ARG;
        if (J.mode != 0) return RG_ERR_UNSUPPORTED;  // ambient occlusion renders one frame at a time
        if (sh.width == 0) sh.width = J.tlas->width;
        if (J.tlas->width != sh.width) return RG_ERR_UNSUPPORTED;  // one traversal width per batch
        if (!rg_trace_depth_ok(J.tlas)) return RG_ERR_UNSUPPORTED;
        int64_t n = (int64_t)J.width * J.height;
        sh.total_pix += n;
        sh.cap += n << J.max_depth;
        for (int k = 0; k <= RG_MAX_DEPTH; ++k) sh.cap_at[k] += n << (k < J.max_depth ? k : J.max_depth);
        sh.n_mats += J.n_mats;
        if (J.max_depth > sh.max_depth) sh.max_depth = J.max_depth;
    }
    if (sh.cap > (1ll << 31) || sh.total_pix > (1ll << 31)) return RG_ERR_UNSUPPORTED;
    return RG_OK;
}

uint64_t batch_bytes(const BatchShape &sh, int32_t n_jobs) {
    RgArena A{nullptr, 0, 0};
    RgWaveBufs b;
    rg_wave_carve(A, sh.total_pix, sh.cap, n_jobs, sh.n_mats, b);
    return A.used;
}

rg_status run_batch(const rg_batch *B, hipStream_t st) {
    RgArena A{(char *)B->scratch, B->scratch_bytes, 0};
    RgWaveBufs b;
    if (!rg_wave_carve(A, B->total_pixels, B->capacity, B->n_jobs, B->n_mats, b)) return RG_ERR_OUT_OF_MEMORY;
    const int64_t total = B->total_pixels;
    k_zero_u64<<<rg_blocks(3 * total, kT), kT, 0, st>>>(b.acc, 3 * total);
    rg_status r = rg_wave_reset(b, st);
    if (r != RG_OK) return r;
    k_camera_batch<<<rg_blocks(total, kT), kT, 0, st>>>(b.jobs, B->n_jobs, total, b.q[0], b.counts + 0);
    RG_LAUNCH_CHECK();
    for (int k = 0; k <= B->max_depth; ++k) {
        r = rg_wave_pass(b, B->width, k, B->cap_at[k], st, RG_TUNE_FRAME, B->has_inst_flags != 0);
        if (r != RG_OK) return r;
    }
    k_resolve_batch<<<rg_blocks(total, kT), kT, 0, st>>>(b.acc, b.jobs, B->n_jobs, total);
    RG_LAUNCH_CHECK();
    return RG_OK;
}

// The two timing events of a call that reports stats, destroyed however the
// call ends.
struct StatEvents {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    StatEvents() = default;
    StatEvents(const StatEvents &) = delete;
    StatEvents &operator=(const StatEvents &) = delete;
    ~StatEvents() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
    rg_status start(hipStream_t st) {
        RG_HIP(hipEventCreate(&e0));
        RG_HIP(hipEventCreate(&e1));
        RG_HIP(hipEventRecord(e0, st));
        return RG_OK;
    }
};

rg_status finish_stats(hipStream_t st, hipEvent_t e0, hipEvent_t e1, const unsigned long long *dstat,
                       rg_render_stats *stats) {
    RG_HIP(hipEventRecord(e1, st));
    unsigned long long hs[2] = {0, 0};
    RG_HIP(hipMemcpyAsync(hs, dstat, 16, hipMemcpyDeviceToHost, st));
    RG_HIP(hipStreamSynchronize(st));
    float ms = 0.0f;
    RG_HIP(hipEventElapsedTime(&ms, e0, e1));
    stats->rays_traced = hs[0];
    stats->shadow_rays = hs[1];
    stats->ms_total = ms;
    return RG_OK;
}

// Copies one pass's queues into a caller's capture buffers: the closest-hit
// rays with their float32 t and their hit as input indices (the record's
// instance, the leaf-order triangle's input index), and the shadow rays with
// their any-hit result; the first `cap` entries of each, and both counts.
struct CaptureArgs {
    RgQueue q;
    const float *hit_t;
    const uint32_t *hit_rec, *hit_slot, *ccount;
    RgShadowQ sq;
    const uint32_t *scount;
    RgTlasRef T;
    int64_t cap;
    int k;
    rg_capture out;
};

__global__ void __launch_bounds__(kT) k_capture(CaptureArgs a) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    const int64_t nc = (int64_t)*a.ccount < a.cap ? (int64_t)*a.ccount : a.cap;
    const int64_t ns = (int64_t)*a.scount < a.cap ? (int64_t)*a.scount : a.cap;
    if (i == 0) {
        a.out.counts[2 * a.k] = *a.ccount;
        a.out.counts[2 * a.k + 1] = *a.scount;
    }
    const uint64_t base = (uint64_t)a.k * a.cap;
    if (i < nc) {
        for (int c = 0; c < 8; ++c) a.out.rays[(8 * (uint64_t)a.k + c) * a.cap + i] = a.q.ray[c][i];
        a.out.t[base + i] = a.hit_t[i];
        const uint32_t rec = a.hit_rec[i];
        uint32_t inst = RG_MISS, prim = RG_MISS;
        if (rec != RG_MISS) {
            const RgInst &R = a.T.recs[rec];
            inst = R.inst;
            prim = reinterpret_cast<const RgTri *>(R.tris)[a.hit_slot[i]].prim;
        }
        a.out.inst[base + i] = inst;
        a.out.prim[base + i] = prim;
    }
    if (i < ns) {
        for (int c = 0; c < 8; ++c) a.out.shadow_rays[(8 * (uint64_t)a.k + c) * a.cap + i] = a.sq.ray[c][i];
        a.out.occluded[base + i] = a.sq.occ[i];
    }
}

}  // namespace

// ------------------------------------------------ wavefront passes
bool rg_wave_carve(RgArena &A, int64_t pixels, int64_t cap, int64_t n_jobs, int64_t n_mats, RgWaveBufs &b) {
    b.acc = A.take<unsigned long long>(3 * pixels);
    b.stat = A.take<unsigned long long>(4);
    b.counts = A.take<uint32_t>(8);
    b.jobs = A.take<RgJobDev>(n_jobs);
    b.tlas = A.take<RgTlasRef>(n_jobs);
    b.mats = A.take<RgMat>(n_mats);
    b.hit_t = A.take<float>(cap);
    b.hit_rec = A.take<uint32_t>(cap);
    b.hit_slot = A.take<uint32_t>(cap);
    for (int k = 0; k < 2; ++k) {
        for (int c = 0; c < 8; ++c) b.q[k].ray[c] = A.take<float>(cap);
        b.q[k].pix = A.take<uint32_t>(cap);
        b.q[k].job = A.take<uint32_t>(cap);
        for (int c = 0; c < 3; ++c) b.q[k].beta[c] = A.take<float>(cap);
    }
    for (int c = 0; c < 8; ++c) b.sq.ray[c] = A.take<float>(cap);
    b.sq.pix = A.take<uint32_t>(cap);
    b.sq.job = A.take<uint32_t>(cap);
    for (int c = 0; c < 3; ++c) b.sq.pend[c] = A.take<float>(cap);
    b.sq.occ = A.take<uint8_t>(cap);
    b.cap = cap;
    return !A.overflow();
}

rg_status rg_wave_reset(const RgWaveBufs &b, hipStream_t st) {
    k_zero_u64<<<1, kT, 0, st>>>(b.stat, 4);
    k_fill_u32<<<1, kT, 0, st>>>(b.counts, 0u, 8);
    RG_LAUNCH_CHECK();
    return RG_OK;
}

rg_status rg_wave_put_job(const RgWaveBufs &b, uint32_t slot, const RgJobDev &J, const RgTlasRef &T,
                          const rg_material *host_mats, int32_t n_mats, hipStream_t st) {
    k_put_job<<<1, 64, 0, st>>>(b.jobs, b.tlas, slot, J, T);
    for (int32_t c = 0; c < n_mats; c += kMatChunk) {
        MatChunk m;
        const int cnt = n_mats - c < kMatChunk ? n_mats - c : kMatChunk;
        memcpy(m.m, host_mats + c, sizeof(RgMat) * (size_t)cnt);
        k_put_mats<<<1, kMatChunk, 0, st>>>(b.mats + J.mat_off + c, m, cnt);
    }
    const int64_t n = 3 * (int64_t)J.width * J.height;
    k_zero_u64<<<rg_blocks(n, kT), kT, 0, st>>>(b.acc + 3 * (uint64_t)J.pix_off, n);
    RG_LAUNCH_CHECK();
    return RG_OK;
}

rg_status rg_wave_camera(const RgWaveBufs &b, uint32_t slot, const RgJobDev &J, int queue, hipStream_t st) {
    const int64_t n = (int64_t)J.width * J.height;
    k_reserve<<<1, 64, 0, st>>>(b.counts + (queue & 1), (uint32_t)n, b.counts + 4);
    k_camera_job<<<rg_blocks(n, kT), kT, 0, st>>>(J, slot, b.q[queue & 1], b.counts + 4, b.cap);
    RG_LAUNCH_CHECK();
    return RG_OK;
}

rg_status rg_wave_pass(const RgWaveBufs &b, int32_t width, int64_t pass, int64_t bound, hipStream_t st,
                       int scope, bool opt, RgShadowSide *side) {
    if (bound < 1) return RG_OK;
    if (bound > b.cap) bound = b.cap;
    const RgQueue &qin = b.q[pass & 1], &qout = b.q[(pass + 1) & 1];
    uint32_t *cin = b.counts + (pass & 1), *cout = b.counts + ((pass + 1) & 1), *csq = b.counts + 2;
    RgTraceArgs tc = {};
    for (int c = 0; c < 8; ++c) tc.ray[c] = qin.ray[c];
    tc.n = bound;
    tc.count = cin;
    tc.ray_job = qin.job;
    tc.jobs = b.tlas;
    tc.t = b.hit_t;
    tc.inst = b.hit_rec;
    tc.prim = b.hit_slot;
    tc.opt = opt;
    rg_status r = rg_trace_launch(width, false, rgt::kRender, tc, st, scope);
    if (r != RG_OK) return r;
    // the shadow queue and its count are reused below: the previous pass's
    // shadow work must be done with them
    if (side && side->pending) RG_HIP(hipStreamWaitEvent(st, side->shadowed, 0));
    k_pass_counts<<<1, 1, 0, st>>>(b.stat, cin, cout, csq);
    ShadeArgs sa;
    sa.in = qin;
    sa.count_in = cin;
    sa.hit_t = b.hit_t;
    sa.hit_rec = b.hit_rec;
    sa.hit_slot = b.hit_slot;
    sa.tlas = b.tlas;
    sa.jobs = b.jobs;
    sa.mats = b.mats;
    sa.pass = pass;
    sa.acc = b.acc;
    sa.out = qout;
    sa.count_out = cout;
    sa.sq = b.sq;
    sa.count_sq = csq;
    sa.cap_out = b.cap;
    sa.cap_sq = b.cap;
    sa.n_max = bound;
    {
        const int64_t want = (int64_t)rg_cu_count() * 3;
        const int64_t need = rg_blocks(bound, kShadeT);
        k_shade<<<(unsigned)(need < want ? need : want), kShadeT, 0, st>>>(sa);
    }
    RG_LAUNCH_CHECK();
    hipStream_t s2 = st;
    if (side) {
        RG_HIP(hipEventRecord(side->shaded, st));
        RG_HIP(hipStreamWaitEvent(side->st, side->shaded, 0));
        s2 = side->st;
    }
    RgTraceArgs ts = {};
    for (int c = 0; c < 8; ++c) ts.ray[c] = b.sq.ray[c];
    ts.n = bound;
    ts.count = csq;
    ts.ray_job = b.sq.job;
    ts.jobs = b.tlas;
    ts.occluded = b.sq.occ;
    ts.opt = opt;
    r = rg_trace_launch(width, true, rgt::kRender, ts, s2, scope);
    if (r != RG_OK) return r;
    k_stat_add<<<1, 1, 0, s2>>>(b.stat + 1, csq);
    k_shadow_resolve<<<rg_blocks(bound, kT), kT, 0, s2>>>(b.sq, csq, b.acc);
    RG_LAUNCH_CHECK();
    if (side) {
        RG_HIP(hipEventRecord(side->shadowed, s2));
        side->pending = true;
    }
    return RG_OK;
}

rg_status rg_wave_resolve(const RgWaveBufs &b, const RgJobDev &J, hipStream_t st) {
    const int64_t n = (int64_t)J.width * J.height;
    k_resolve_job<<<rg_blocks(3 * n, kT), kT, 0, st>>>(b.acc + 3 * (uint64_t)J.pix_off, n, J.image);
    RG_LAUNCH_CHECK();
    return RG_OK;
}

extern "C" {

rg_status rg_camera_rays(const rg_camera *cam, int32_t width, int32_t height, float *const rays[8], void *stream) {
    if (!cam || !rays || width < 1 || height < 1 || (int64_t)width * height > (1ll << 31)) return RG_ERR_INVALID_ARG;
    for (int k = 0; k < 8; ++k)
        if (!rays[k]) return RG_ERR_INVALID_ARG;
    int64_t n = (int64_t)width * height;
    k_camera_rays<<<rg_blocks(n, kT), kT, 0, (hipStream_t)stream>>>(
        *cam, width, height, rays[0], rays[1], rays[2], rays[3], rays[4], rays[5], rays[6], rays[7]);
    RG_LAUNCH_CHECK();
    return rg_debug_done(RG_OK, (hipStream_t)stream);
}

rg_status rg_ao_rays_scratch(int64_t n, uint64_t *scratch_bytes) {
    if (n < 0 || !scratch_bytes) return RG_ERR_INVALID_ARG;
    *scratch_bytes = ((uint64_t)rg_blocks(n, kT) * 4u + 255u) & ~uint64_t(255);
    return RG_OK;
}

rg_status rg_ao_rays(const rg_tlas *tlas, rg_rays rays, int64_t n, const uint32_t *hit_inst, const uint32_t *hit_prim,
                     const float *hit_t, uint64_t seed, float ao_tmax, float *const out_rays[8], uint32_t *out_src,
                     uint32_t *out_count, void *scratch, uint64_t scratch_bytes, void *stream) {
    if (!tlas_valid(tlas) || n < 1 || n > (1ll << 28) || !hit_inst || !hit_prim || !hit_t || !out_rays || !out_src ||
        !out_count || !scratch)
        return RG_ERR_INVALID_ARG;
    if (!rays.ox || !rays.oy || !rays.oz || !rays.dx || !rays.dy || !rays.dz) return RG_ERR_INVALID_ARG;
    for (int k = 0; k < 8; ++k)
        if (!out_rays[k]) return RG_ERR_INVALID_ARG;
    uint64_t need;
    rg_ao_rays_scratch(n, &need);
    if (scratch_bytes < need) return RG_ERR_OUT_OF_MEMORY;
    AoArgs a = {};
    a.ray[0] = rays.ox; a.ray[1] = rays.oy; a.ray[2] = rays.oz;
    a.ray[3] = rays.dx; a.ray[4] = rays.dy; a.ray[5] = rays.dz;
    a.n = n;
    a.hit_a = hit_inst;
    a.hit_b = hit_prim;
    a.hit_t = hit_t;
    a.rec_of = (const uint32_t *)((const char *)tlas->buf + tlas->rec_off);
    a.recs = (const RgInst *)((const char *)tlas->buf + tlas->inst_off);
    a.seed = seed;
    a.tmax = ao_tmax;
    for (int k = 0; k < 8; ++k) a.out[k] = out_rays[k];
    a.src = out_src;
    a.count = out_count;
    a.block_off = (uint32_t *)scratch;
    a.map = true;
    return rg_debug_done(ao_generate(a, (hipStream_t)stream), (hipStream_t)stream);
}

rg_status rg_batch_sizes(const rg_job *jobs, int32_t n_jobs, uint64_t *scratch_bytes) {
    if (!scratch_bytes) return RG_ERR_INVALID_ARG;
    BatchShape sh;
    rg_status r = batch_shape(jobs, n_jobs, sh);
    if (r != RG_OK) return r;
    *scratch_bytes = batch_bytes(sh, n_jobs);
    return RG_OK;
}

rg_status rg_batch_prepare(const rg_job *jobs, int32_t n_jobs, void *scratch, uint64_t scratch_bytes, void *stream,
                           rg_batch *out) {
    if (!scratch || !out) return RG_ERR_INVALID_ARG;
    BatchShape sh;
    rg_status r = batch_shape(jobs, n_jobs, sh);
    if (r != RG_OK) return r;
    if (scratch_bytes < batch_bytes(sh, n_jobs)) return RG_ERR_OUT_OF_MEMORY;
    std::vector<RgJobDev> hj((size_t)n_jobs);
    std::vector<RgTlasRef> ht((size_t)n_jobs);
    std::vector<RgMat> hm((size_t)sh.n_mats);
    rg_batch B = {};
    uint32_t pix = 0, mo = 0;
    for (int32_t j = 0; j < n_jobs; ++j) {
        const rg_job &J = jobs[j];
        hj[j].cam = J.cam;
        hj[j].light = J.light;
        hj[j].pix_off = pix;
        hj[j].width = (uint32_t)J.width;
        hj[j].height = (uint32_t)J.height;
        hj[j].mat_off = mo;
        hj[j].n_mats = (uint32_t)J.n_mats;
        hj[j].max_depth = J.max_depth;
        hj[j].start = 0;
        hj[j].image = J.image;
        ht[j].nodes = (const char *)J.tlas->buf + J.tlas->nodes_off;
        ht[j].recs = (const RgInst *)((const char *)J.tlas->buf + J.tlas->inst_off);
        if (J.tlas->has_inst_flags) B.has_inst_flags = 1;
        memcpy(&hm[mo], J.mats, sizeof(RgMat) * (size_t)J.n_mats);
        pix += (uint32_t)(J.width * J.height);
        mo += (uint32_t)J.n_mats;
    }
    B.scratch = scratch;
    B.scratch_bytes = scratch_bytes;
    B.n_jobs = n_jobs;
    B.width = sh.width;
    B.max_depth = sh.max_depth;
    B.n_mats = sh.n_mats;
    B.total_pixels = sh.total_pix;
    B.capacity = sh.cap;
    for (int k = 0; k <= RG_MAX_DEPTH; ++k) B.cap_at[k] = sh.cap_at[k];
    RgArena A{(char *)scratch, scratch_bytes, 0};
    RgWaveBufs b;
    if (!rg_wave_carve(A, sh.total_pix, sh.cap, n_jobs, sh.n_mats, b)) return RG_ERR_OUT_OF_MEMORY;
    hipStream_t st = (hipStream_t)stream;
    RG_HIP(hipMemcpyAsync(b.jobs, hj.data(), sizeof(RgJobDev) * hj.size(), hipMemcpyHostToDevice, st));
    RG_HIP(hipMemcpyAsync(b.tlas, ht.data(), sizeof(RgTlasRef) * ht.size(), hipMemcpyHostToDevice, st));
    RG_HIP(hipMemcpyAsync(b.mats, hm.data(), sizeof(RgMat) * hm.size(), hipMemcpyHostToDevice, st));
    RG_HIP(hipStreamSynchronize(st));  // the host tables may go away once this returns
    *out = B;
    return RG_OK;
}

static rg_status batch_impl(const rg_batch *batch, void *stream, rg_render_stats *stats);

rg_status rg_batch_render(const rg_batch *batch, void *stream, rg_render_stats *stats) {
    return rg_debug_done(batch_impl(batch, stream, stats), (hipStream_t)stream);
}

static rg_status batch_impl(const rg_batch *batch, void *stream, rg_render_stats *stats) {
    if (!batch || !batch->scratch || batch->n_jobs < 1) return RG_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    StatEvents ev;
    if (stats) {
        const rg_status re = ev.start(st);
        if (re != RG_OK) return re;
    }
    rg_status r = run_batch(batch, st);
    if (r != RG_OK) return r;
    if (stats) {
        RgArena A{(char *)batch->scratch, batch->scratch_bytes, 0};
        RgWaveBufs b;
        rg_wave_carve(A, batch->total_pixels, batch->capacity, batch->n_jobs, batch->n_mats, b);
        return finish_stats(st, ev.e0, ev.e1, b.stat, stats);
    }
    return RG_OK;
}

rg_status rg_render_sizes(int32_t width, int32_t height, int32_t max_depth, int32_t mode, uint64_t *scratch_bytes) {
    if (!scratch_bytes || width < 1 || height < 1 || max_depth < 0 || max_depth > RG_MAX_DEPTH ||
        (mode != 0 && mode != 1))
        return RG_ERR_INVALID_ARG;
    int64_t n = (int64_t)width * height;
    if ((n << (mode == 1 ? 3 : max_depth)) > (1ll << 31)) return RG_ERR_UNSUPPORTED;
    RgArena A{nullptr, 0, 0};
    if (mode == 1) {
        AoBufs b;
        carve_ao(A, n, b);
    } else {
        RgWaveBufs b;
        rg_wave_carve(A, n, n << max_depth, 1, 256, b);
    }
    *scratch_bytes = A.used;
    return RG_OK;
}

rg_status rg_render(const rg_tlas *tlas, const rg_material *mats, int32_t n_mats, const rg_camera *cam,
                    const rg_light *light, int32_t width, int32_t height, int32_t max_depth, int32_t mode,
                    uint64_t seed, float *image, void *scratch, uint64_t scratch_bytes, void *stream,
                    rg_render_stats *stats) {
    return rg_render_ex(tlas, mats, n_mats, cam, light, width, height, max_depth, mode, seed, image, nullptr,
                        scratch, scratch_bytes, stream, stats);
}

static rg_status render_impl(const rg_tlas *tlas, const rg_material *mats, int32_t n_mats, const rg_camera *cam,
                             const rg_light *light, int32_t width, int32_t height, int32_t max_depth, int32_t mode,
                             uint64_t seed, float *image, uint32_t *primary_mat, void *scratch,
                             uint64_t scratch_bytes, void *stream, rg_render_stats *stats,
                             const rg_capture *capture = nullptr);

rg_status rg_render_ex(const rg_tlas *tlas, const rg_material *mats, int32_t n_mats, const rg_camera *cam,
                       const rg_light *light, int32_t width, int32_t height, int32_t max_depth, int32_t mode,
                       uint64_t seed, float *image, uint32_t *primary_mat, void *scratch, uint64_t scratch_bytes,
                       void *stream, rg_render_stats *stats) {
    return rg_debug_done(render_impl(tlas, mats, n_mats, cam, light, width, height, max_depth, mode, seed, image,
                                     primary_mat, scratch, scratch_bytes, stream, stats),
                         (hipStream_t)stream);
}

rg_status rg_render_capture(const rg_tlas *tlas, const rg_material *mats, int32_t n_mats, const rg_camera *cam,
                            const rg_light *light, int32_t width, int32_t height, int32_t max_depth, uint64_t seed,
                            float *image, void *scratch, uint64_t scratch_bytes, const rg_capture *capture,
                            void *stream) {
    if (!capture || capture->capacity < 1 || !capture->rays || !capture->t || !capture->inst || !capture->prim ||
        !capture->shadow_rays || !capture->occluded || !capture->counts)
        return RG_ERR_INVALID_ARG;
    return rg_debug_done(render_impl(tlas, mats, n_mats, cam, light, width, height, max_depth, 0, seed, image,
                                     nullptr, scratch, scratch_bytes, stream, nullptr, capture),
                         (hipStream_t)stream);
}

static rg_status render_impl(const rg_tlas *tlas, const rg_material *mats, int32_t n_mats, const rg_camera *cam,
                             const rg_light *light, int32_t width, int32_t height, int32_t max_depth, int32_t mode,
                             uint64_t seed, float *image, uint32_t *primary_mat, void *scratch,
                             uint64_t scratch_bytes, void *stream, rg_render_stats *stats,
                             const rg_capture *capture) {
    if (!tlas_valid(tlas) || !mats || n_mats < 1 || n_mats > 256 || !cam || !light || !image || !scratch)
        return RG_ERR_INVALID_ARG;
    if (primary_mat && mode != 0) return RG_ERR_UNSUPPORTED;
    uint64_t need = 0;
    rg_status r = rg_render_sizes(width, height, max_depth, mode, &need);
    if (r != RG_OK) return r;
    if (scratch_bytes < need) return RG_ERR_OUT_OF_MEMORY;
    if (!rg_trace_depth_ok(tlas)) return RG_ERR_UNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    if (mode == 0) {
        // one frame: the record goes in through kernel arguments, so the
        // whole frame is launches only (no host wait unless stats)
        const int64_t n = (int64_t)width * height;
        RgArena A{(char *)scratch, scratch_bytes, 0};
        RgWaveBufs b;
        if (!rg_wave_carve(A, n, n << max_depth, 1, 256, b)) return RG_ERR_OUT_OF_MEMORY;
        StatEvents ev;
        if (stats) {
            const rg_status re = ev.start(st);
            if (re != RG_OK) return re;
        }
        RgJobDev J = {};
        J.cam = *cam;
        J.light = *light;
        J.width = (uint32_t)width;
        J.height = (uint32_t)height;
        J.n_mats = (uint32_t)n_mats;
        J.max_depth = max_depth;
        J.image = image;
        J.gbuf = primary_mat;
        RgTlasRef T = {(const char *)tlas->buf + tlas->nodes_off,
                       (const RgInst *)((const char *)tlas->buf + tlas->inst_off)};
        if ((r = rg_wave_reset(b, st)) != RG_OK) return r;
        if ((r = rg_wave_put_job(b, 0, J, T, mats, n_mats, st)) != RG_OK) return r;
        if ((r = rg_wave_camera(b, 0, J, 0, st)) != RG_OK) return r;
        for (int k = 0; k <= max_depth; ++k) {
            if ((r = rg_wave_pass(b, tlas->width, k, n << k, st, RG_TUNE_FRAME, tlas->has_inst_flags != 0)) != RG_OK)
                return r;
            if (capture) {
                // pass k's queues, before pass k + 1 reuses them
                CaptureArgs ca;
                ca.q = b.q[k & 1];
                ca.hit_t = b.hit_t;
                ca.hit_rec = b.hit_rec;
                ca.hit_slot = b.hit_slot;
                ca.ccount = b.counts + (k & 1);
                ca.sq = b.sq;
                ca.scount = b.counts + 2;
                ca.T = T;
                ca.cap = capture->capacity;
                ca.k = k;
                ca.out = *capture;
                const int64_t m = (n << k) < capture->capacity ? (n << k) : capture->capacity;
                k_capture<<<rg_blocks(m, kT), kT, 0, st>>>(ca);
                RG_LAUNCH_CHECK();
            }
        }
        if ((r = rg_wave_resolve(b, J, st)) != RG_OK) return r;
        if (stats) return finish_stats(st, ev.e0, ev.e1, b.stat, stats);
        return RG_OK;
    }
    const int64_t n = (int64_t)width * height;
    RgArena A{(char *)scratch, scratch_bytes, 0};
    AoBufs b;
    if (!carve_ao(A, n, b)) return RG_ERR_OUT_OF_MEMORY;
    StatEvents ev;
    if (stats) {
        const rg_status re = ev.start(st);
        if (re != RG_OK) return re;
    }
    k_zero_u64<<<rg_blocks(3 * n, kT), kT, 0, st>>>(b.acc, 3 * n);
    k_zero_u64<<<1, kT, 0, st>>>(b.stat, 4);
    k_fill_u32<<<1, kT, 0, st>>>(b.counts, 0u, 8);
    k_camera_rays<<<rg_blocks(n, kT), kT, 0, st>>>(*cam, width, height, b.cam[0], b.cam[1], b.cam[2], b.cam[3],
                                                   b.cam[4], b.cam[5], b.cam[6], b.cam[7]);
    RG_LAUNCH_CHECK();
    RgTraceArgs ta = trace_args(tlas);
    for (int c = 0; c < 8; ++c) ta.ray[c] = b.cam[c];
    ta.n = n;
    ta.t = b.hit_t;
    ta.inst = b.hit_rec;
    ta.prim = b.hit_slot;
    r = rg_trace_launch(tlas->width, false, rgt::kRender, ta, st, RG_TUNE_FRAME);
    if (r != RG_OK) return r;
    AoArgs a = {};
    for (int c = 0; c < 6; ++c) a.ray[c] = b.cam[c];
    a.n = n;
    a.hit_a = b.hit_rec;
    a.hit_b = b.hit_slot;
    a.hit_t = b.hit_t;
    a.recs = ta.recs;
    a.seed = seed;
    a.tmax = 5.0f;
    for (int c = 0; c < 8; ++c) a.out[c] = b.ao_ray[c];
    a.src = b.ao_src;
    a.count = b.counts + 2;
    a.block_off = b.ao_blk;
    a.map = false;
    r = ao_generate(a, st);
    if (r != RG_OK) return r;
    RgTraceArgs tb = trace_args(tlas);
    for (int c = 0; c < 8; ++c) tb.ray[c] = b.ao_ray[c];
    tb.n = 8 * n;
    tb.count = b.counts + 2;
    tb.occluded = b.ao_occ;
    r = rg_trace_launch(tlas->width, true, rgt::kRender, tb, st, RG_TUNE_FRAME);
    if (r != RG_OK) return r;
    k_ao_accum<<<rg_blocks(8 * n, kT), kT, 0, st>>>(b.ao_occ, b.ao_src, b.counts + 2, b.acc);
    k_ao_resolve<<<rg_blocks(n, kT), kT, 0, st>>>(b.acc, b.hit_rec, n, image);
    RG_LAUNCH_CHECK();
    k_stat_add<<<1, 1, 0, st>>>(b.stat, b.counts + 0);
    k_stat_add<<<1, 1, 0, st>>>(b.stat + 1, b.counts + 2);
    if (stats) return finish_stats(st, ev.e0, ev.e1, b.stat, stats);
    return RG_OK;
}

}  // extern "C"

// ------------------------------------------------ rg_render_static
// Scratch memory of rg_render_static: a device array of RG_STATIC_SCRATCH_BYTES
// in the library's code object.  Each GPU the library runs on holds its own
// copy, from the module's load on that device until the process ends.  Host
// code never uses the array's name as an address (on the host it names a
// stand-in, not device memory): the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[RG_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices] = {};

rg_status static_scratch(void **out) {
    int dev = 0;
    RG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return RG_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        RG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return RG_ERR_HIP;
        g_static_ptr[dev] = p;
    }
    *out = g_static_ptr[dev];
    return RG_OK;
}
}  // namespace

extern "C" rg_status rg_render_static(const rg_tlas *tlas, const rg_material *mats, int32_t n_mats,
                                      const rg_camera *cam, const rg_light *light, int32_t width, int32_t height,
                                      int32_t max_depth, int32_t mode, uint64_t seed, float *image, void *stream) {
    uint64_t need = 0;
    rg_status r = rg_render_sizes(width, height, max_depth, mode, &need);
    if (r != RG_OK) return r;
    if (need > RG_STATIC_SCRATCH_BYTES) {
        rg_set_error(__FILE__, __LINE__, "rg_render_static: frame needs more scratch than RG_STATIC_SCRATCH_BYTES");
        return RG_ERR_OUT_OF_MEMORY;
    }
    void *p = nullptr;
    if ((r = static_scratch(&p)) != RG_OK) return r;
    // the same passes as rg_render; every counter, statistic and accumulator
    // that must start at zero is cleared by the passes' own fill kernels
    return rg_render_ex(tlas, mats, n_mats, cam, light, width, height, max_depth, mode, seed, image, nullptr, p,
                        RG_STATIC_SCRATCH_BYTES, stream, nullptr);
}
