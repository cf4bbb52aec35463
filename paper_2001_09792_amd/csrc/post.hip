// post.hip -- the frame's post-process passes (section 2.1: the engine's
// compute system runs a screen-space roughness approximation and fast
// approximate anti-aliasing on the traced image).
//
// Roughness blur: a material-aware Gaussian whose width follows the
// roughness of the material seen at the pixel, as two 1-D passes (x, then y)
// over the taps -R..R with weights exp(-k^2 / (2 sigma^2)), sigma = r R / 3,
// counting only taps inside the image that show the centre's material and
// normalising over them.  FXAA: Lottes' method (2009, "quality" variant) on
// the perceptual luma sqrt(clamp(0.299 R + 0.587 G + 0.114 B, 0, 1)).
//
// Both are memory-bound stencils over float[h][w][3] images: one thread per
// pixel, 64 x 4 pixel blocks, so that a wave reads one row segment; the blur
// stages each block's pixels and their halo along its axis in LDS.
#include "rg_internal.h"

namespace {

constexpr int kBX = 64, kBY = 4;
constexpr float kRoughMin = 1.0f / 256.0f;
constexpr float kEdgeRel = 0.125f, kEdgeMin = 0.0625f, kSubpix = 0.75f;
constexpr int kSteps = 12;
__constant__ float c_steps[kSteps] = {1.0f, 1.0f, 1.0f, 1.0f, 1.0f, 1.5f, 2.0f, 2.0f, 2.0f, 2.0f, 4.0f, 8.0f};

struct Px3 {
    float r, g, b;
};
__device__ inline Px3 ld3(const float *__restrict__ img, int64_t p) {
    return {img[3 * p], img[3 * p + 1], img[3 * p + 2]};
}
__device__ inline void st3(float *__restrict__ img, int64_t p, Px3 v) {
    img[3 * p] = v.r;
    img[3 * p + 1] = v.g;
    img[3 * p + 2] = v.b;
}

// One pass of the blur along x (AXIS 0) or y (AXIS 1).  The block's pixels
// and the `radius` pixels beyond them along the axis are staged in LDS once,
// each as (r, g, b, material bits) in 16 bytes, so a tap is one LDS read.
constexpr uint32_t kOutside = 0xFFFFFFFEu;  // material of positions outside the image

template <int AXIS>
__global__ void __launch_bounds__(kBX *kBY) k_blur(const float *__restrict__ in, const uint32_t *__restrict__ mat,
                                                   const float *__restrict__ rough, uint32_t n_mats, int w, int h,
                                                   int radius, float *__restrict__ out) {
    extern __shared__ float4 tile[];
    const int tid = threadIdx.y * kBX + threadIdx.x;
    const int x0 = blockIdx.x * kBX, y0 = blockIdx.y * kBY;
    const int x = x0 + threadIdx.x, y = y0 + threadIdx.y;
    const bool inside = x < w && y < h;
    const int64_t p = (int64_t)y * w + x;
    const uint32_t m = inside ? mat[p] : kOutside;
    float r = 0.0f;
    if (m < n_mats) r = fminf(fmaxf(rough[m], 0.0f), 1.0f);
    // sky, unknown material, smooth, NaN roughness or no window: a copy; a
    // block without any pixel to blur stages nothing
    const bool blur = inside && r >= kRoughMin && radius > 0;
    if (!__syncthreads_or(blur)) {
        if (inside) st3(out, p, ld3(in, p));
        return;
    }
    const int TW = AXIS == 0 ? kBX + 2 * radius : kBX, TH = AXIS == 0 ? kBY : kBY + 2 * radius;
    const int gx0 = AXIS == 0 ? x0 - radius : x0, gy0 = AXIS == 0 ? y0 : y0 - radius;
    for (int i = tid; i < TW * TH; i += kBX * kBY) {
        const int gx = gx0 + i % TW, gy = gy0 + i / TW;
        float4 v = make_float4(0.0f, 0.0f, 0.0f, __uint_as_float(kOutside));
        if (gx >= 0 && gx < w && gy >= 0 && gy < h) {
            const int64_t q = (int64_t)gy * w + gx;
            v = make_float4(in[3 * q], in[3 * q + 1], in[3 * q + 2], __uint_as_float(mat[q]));
        }
        tile[i] = v;
    }
    __syncthreads();
    if (!inside) return;
    const int c = AXIS == 0 ? threadIdx.y * TW + threadIdx.x + radius : (threadIdx.y + radius) * TW + threadIdx.x;
    const int step = AXIS == 0 ? 1 : TW;
    const float4 c0 = tile[c];
    if (!blur) {
        st3(out, p, {c0.x, c0.y, c0.z});
        return;
    }
    const float sigma = r * (float)radius / 3.0f;
    const float inv = 1.0f / (2.0f * sigma * sigma);
    float nr = c0.x, ng = c0.y, nb = c0.z, den = 1.0f;  // the centre tap, weight 1
    // taps -k and +k share their weight: one exponential per distance
    for (int k = 1; k <= radius; ++k) {
        const float wt = expf(-(float)(k * k) * inv);
        const float4 a = tile[c - k * step], b = tile[c + k * step];
        if (__float_as_uint(a.w) == m) {
            nr += wt * a.x;
            ng += wt * a.y;
            nb += wt * a.z;
            den += wt;
        }
        if (__float_as_uint(b.w) == m) {
            nr += wt * b.x;
            ng += wt * b.y;
            nb += wt * b.z;
            den += wt;
        }
    }
    const float s = 1.0f / den;  // den >= 1
    st3(out, p, {nr * s, ng * s, nb * s});
}

__global__ void __launch_bounds__(kBX *kBY) k_luma(const float *__restrict__ in, int w, int h,
                                                   float *__restrict__ luma) {
    const int x = blockIdx.x * kBX + threadIdx.x, y = blockIdx.y * kBY + threadIdx.y;
    if (x >= w || y >= h) return;
    const int64_t p = (int64_t)y * w + x;
    const Px3 c = ld3(in, p);
    const float v = 0.299f * c.r + 0.587f * c.g + 0.114f * c.b;
    luma[p] = sqrtf(fminf(fmaxf(v, 0.0f), 1.0f));
}

struct LumaImg {
    const float *__restrict__ l;
    int w, h;
    __device__ inline float at(int x, int y) const {
        x = x < 0 ? 0 : (x >= w ? w - 1 : x);
        y = y < 0 ? 0 : (y >= h ? h - 1 : y);
        return l[(int64_t)y * w + x];
    }
    // bilinear, pixel centres at integer coordinates, clamped at the borders
    __device__ inline float bilinear(float px, float py) const {
        const float x0 = floorf(px), y0 = floorf(py);
        const float fx = px - x0, fy = py - y0;
        const int xi = (int)x0, yi = (int)y0;
        const float top = (1.0f - fx) * at(xi, yi) + fx * at(xi + 1, yi);
        const float bot = (1.0f - fx) * at(xi, yi + 1) + fx * at(xi + 1, yi + 1);
        return (1.0f - fy) * top + fy * bot;
    }
};

__global__ void __launch_bounds__(kBX *kBY) k_fxaa(const float *__restrict__ in, const float *__restrict__ luma,
                                                   int w, int h, float *__restrict__ out) {
    const int x = blockIdx.x * kBX + threadIdx.x, y = blockIdx.y * kBY + threadIdx.y;
    if (x >= w || y >= h) return;
    const int64_t p = (int64_t)y * w + x;
    const LumaImg L{luma, w, h};
    const float m = luma[p], n = L.at(x, y - 1), s = L.at(x, y + 1), wl = L.at(x - 1, y), e = L.at(x + 1, y);
    const float hi = fmaxf(fmaxf(fmaxf(m, n), fmaxf(s, wl)), e);
    const float lo = fminf(fminf(fminf(m, n), fminf(s, wl)), e);
    const float range = hi - lo;
    if (range < fmaxf(kEdgeMin, hi * kEdgeRel)) {  // too little contrast: no edge here
        st3(out, p, ld3(in, p));
        return;
    }
    const float nw = L.at(x - 1, y - 1), ne = L.at(x + 1, y - 1), sw = L.at(x - 1, y + 1), se = L.at(x + 1, y + 1);
    const float edge_h = fabsf(nw - 2.0f * wl + sw) + 2.0f * fabsf(n - 2.0f * m + s) + fabsf(ne - 2.0f * e + se);
    const float edge_v = fabsf(nw - 2.0f * n + ne) + 2.0f * fabsf(wl - 2.0f * m + e) + fabsf(sw - 2.0f * s + se);
    const bool horiz = edge_h >= edge_v;
    const float l1 = horiz ? n : wl, l2 = horiz ? s : e;
    const float g1 = fabsf(l1 - m), g2 = fabsf(l2 - m);
    const bool first = g1 >= g2;
    const float sign = first ? -1.0f : 1.0f;
    const float lavg = first ? 0.5f * (l1 + m) : 0.5f * (l2 + m);
    const float gscaled = 0.25f * fmaxf(g1, g2);
    // along the edge (ex, ey), across it (px, py)
    const float ex = horiz ? 1.0f : 0.0f, ey = horiz ? 0.0f : 1.0f;
    const float cx = (float)x + 0.5f * sign * (1.0f - ex), cy = (float)y + 0.5f * sign * (1.0f - ey);
    float dist[2], dend[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const float dir = side == 0 ? -1.0f : 1.0f;
        float t = 0.0f, d = 0.0f;
        for (int k = 0; k < kSteps; ++k) {
            t += c_steps[k];
            d = L.bilinear(cx + dir * t * ex, cy + dir * t * ey) - lavg;
            if (fabsf(d) >= gscaled) break;
        }
        dist[side] = t;
        dend[side] = d;
    }
    const bool near_neg = dist[0] < dist[1];
    const float dmin = near_neg ? dist[0] : dist[1];
    const float d_end = near_neg ? dend[0] : dend[1];
    const bool good = (d_end < 0.0f) != ((m - lavg) < 0.0f);
    const float off_edge = good ? 0.5f - dmin / (dist[0] + dist[1]) : 0.0f;
    const float avg = (2.0f * (n + s + wl + e) + (nw + ne + sw + se)) / 12.0f;
    const float sub1 = fminf(fmaxf(fabsf(avg - m) / range, 0.0f), 1.0f);
    const float sub2 = (-2.0f * sub1 + 3.0f) * sub1 * sub1;
    const float off = fmaxf(off_edge, sub2 * sub2 * kSubpix);
    int nx = x + (horiz ? 0 : (int)sign), ny = y + (horiz ? (int)sign : 0);
    nx = nx < 0 ? 0 : (nx >= w ? w - 1 : nx);
    ny = ny < 0 ? 0 : (ny >= h ? h - 1 : ny);
    const Px3 c = ld3(in, p), q = ld3(in, (int64_t)ny * w + nx);
    st3(out, p, {(1.0f - off) * c.r + off * q.r, (1.0f - off) * c.g + off * q.g, (1.0f - off) * c.b + off * q.b});
}

bool size_ok(int32_t w, int32_t h) { return w >= 1 && h >= 1 && (int64_t)w * h <= (1ll << 30); }

uint64_t round_up(uint64_t v) { return (v + 255u) & ~(uint64_t)255u; }

// true when [a, a + na) and [b, b + nb) share a byte
bool overlap(const void *a, uint64_t na, const void *b, uint64_t nb) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

dim3 grid_of(int32_t w, int32_t h) { return dim3((unsigned)((w + kBX - 1) / kBX), (unsigned)((h + kBY - 1) / kBY)); }

}  // namespace

extern "C" {

rg_status rg_post_sizes(int32_t width, int32_t height, uint64_t *scratch_bytes) {
    if (!scratch_bytes || !size_ok(width, height)) return RG_ERR_INVALID_ARG;
    const uint64_t n = (uint64_t)width * (uint64_t)height;
    *scratch_bytes = round_up(12 * n) + round_up(4 * n);
    return RG_OK;
}

rg_status rg_roughness_blur(const float *in, const uint32_t *mat, const float *roughness, int32_t n_mats,
                            int32_t width, int32_t height, int32_t radius, float *out, void *scratch,
                            uint64_t scratch_bytes, void *stream) {
    if (!in || !mat || !roughness || !out || !scratch || n_mats < 1 || radius < 0 ||
        radius > RG_BLUR_RADIUS_MAX || !size_ok(width, height))
        return RG_ERR_INVALID_ARG;
    const uint64_t n = (uint64_t)width * (uint64_t)height;
    uint64_t need = 0;
    rg_post_sizes(width, height, &need);
    if (scratch_bytes < need) return RG_ERR_OUT_OF_MEMORY;
    float *tmp = (float *)scratch;
    if (overlap(in, 12 * n, out, 12 * n) || overlap(tmp, 12 * n, in, 12 * n) || overlap(tmp, 12 * n, out, 12 * n))
        return RG_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const dim3 g = grid_of(width, height), b(kBX, kBY);
    const size_t lds_x = sizeof(float4) * (size_t)(kBX + 2 * radius) * kBY;
    const size_t lds_y = sizeof(float4) * (size_t)kBX * (kBY + 2 * radius);
    k_blur<0><<<g, b, lds_x, st>>>(in, mat, roughness, (uint32_t)n_mats, width, height, radius, tmp);
    k_blur<1><<<g, b, lds_y, st>>>(tmp, mat, roughness, (uint32_t)n_mats, width, height, radius, out);
    RG_LAUNCH_CHECK();
    return rg_debug_done(RG_OK, st);
}

rg_status rg_fxaa(const float *in, int32_t width, int32_t height, float *out, void *scratch, uint64_t scratch_bytes,
                  void *stream) {
    if (!in || !out || !scratch || !size_ok(width, height)) return RG_ERR_INVALID_ARG;
    const uint64_t n = (uint64_t)width * (uint64_t)height;
    uint64_t need = 0;
    rg_post_sizes(width, height, &need);
    if (scratch_bytes < need) return RG_ERR_OUT_OF_MEMORY;
    float *luma = (float *)((char *)scratch + round_up(12 * n));
    if (overlap(in, 12 * n, out, 12 * n) || overlap(luma, 4 * n, in, 12 * n) || overlap(luma, 4 * n, out, 12 * n))
        return RG_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const dim3 g = grid_of(width, height), b(kBX, kBY);
    k_luma<<<g, b, 0, st>>>(in, width, height, luma);
    k_fxaa<<<g, b, 0, st>>>(in, luma, width, height, out);
    RG_LAUNCH_CHECK();
    return rg_debug_done(RG_OK, st);
}

}  // extern "C"
